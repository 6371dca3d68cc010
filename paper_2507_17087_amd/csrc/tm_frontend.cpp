// Front end: translates an IndexTaskMap mapper written in the mapping language
// (the syntax figure of Sec. 7; examples in Fig. 1 and App. A.1) into a
// tm_candidate for a given launch domain and machine.
//
// The launch domain and Machine(GPU) are known at translation time, so every value
// the mapper computes is a concrete integer except the index point.  Index-point
// components are carried symbolically through the only forms a mapping function
// can return as processor coordinates: ip[d] * s / ispace[d] (BLOCK, Fig. 1 and
// Fig. 3) and ip[d] % s (CYCLIC, App. A.1).  Processor-space methods record the
// transformation chain (Fig. 6); decompose(i, domain) takes its factors from
// decompose's argmin over that domain (Sec. 4.2).  Anything else is reported with
// its line and column.
#include <cctype>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "tm_internal.h"

namespace {

// ------------------------------------------------------------------ tokens

enum TokKind { T_NAME, T_INT, T_OP, T_END };

struct Tok {
    TokKind kind;
    std::string text;
    int64_t value = 0;
    int line = 0, col = 0;
};

struct Line {
    int indent = 0;
    int number = 0;
    std::vector<Tok> toks;
};

struct FrontError {
    int line, col;
    std::string msg;
};

[[noreturn]] void fail(const Tok& t, const std::string& msg) { throw FrontError{t.line, t.col, msg}; }

// Logical lines: comments dropped, lines joined while brackets are open.
std::vector<Line> tokenize(const char* src) {
    std::vector<Line> lines;
    Line cur;
    bool have = false;
    int depth = 0, lineno = 1, col = 1;
    const char* p = src;
    bool at_start = true;
    int indent = 0;
    auto flush = [&]() {
        if (have && !cur.toks.empty()) lines.push_back(cur);
        cur = Line{};
        have = false;
    };
    while (*p) {
        const char c = *p;
        if (at_start) {
            indent = 0;
            while (*p == ' ' || *p == '\t') {
                indent += *p == '\t' ? 4 : 1;
                ++p;
                ++col;
            }
            at_start = false;
            continue;
        }
        if (c == '#') {
            while (*p && *p != '\n') ++p;
            continue;
        }
        if (c == '\n') {
            ++p;
            ++lineno;
            col = 1;
            if (depth == 0) flush();
            at_start = depth == 0;
            if (depth > 0) at_start = false;
            continue;
        }
        if (c == ' ' || c == '\t' || c == '\r') {
            ++p;
            ++col;
            continue;
        }
        if (!have) {
            cur.indent = indent;
            cur.number = lineno;
            have = true;
        }
        Tok t;
        t.line = lineno;
        t.col = col;
        if (std::isalpha((unsigned char)c) || c == '_') {
            const char* s = p;
            while (std::isalnum((unsigned char)*p) || *p == '_') ++p;
            t.kind = T_NAME;
            t.text.assign(s, p);
        } else if (std::isdigit((unsigned char)c)) {
            const char* s = p;
            int64_t v = 0;
            while (std::isdigit((unsigned char)*p)) {
                if (v > (INT64_MAX - 9) / 10) fail(t, "integer literal too large");
                v = v * 10 + (*p - '0');
                ++p;
            }
            t.kind = T_INT;
            t.text.assign(s, p);
            t.value = v;
        } else {
            static const char* two[] = {"==", "!=", "<=", ">=", "//"};
            t.kind = T_OP;
            bool done = false;
            for (const char* op : two)
                if (p[0] == op[0] && p[1] == op[1]) {
                    t.text = op;
                    p += 2;
                    done = true;
                    break;
                }
            if (!done) {
                if (!std::strchr("()[],.:*/%+-=?<>", c)) fail(t, std::string("unexpected character '") + c + "'");
                t.text = std::string(1, c);
                ++p;
                if (c == '(' || c == '[') ++depth;
                if ((c == ')' || c == ']') && depth > 0) --depth;
            }
        }
        col += (int)t.text.size();
        cur.toks.push_back(t);
    }
    flush();
    return lines;
}

// ------------------------------------------------------------------ values

// A scalar: a constant, or a function of one index-point component.
struct Scalar {
    enum Kind { CONST, IP, IPMUL, BLOCK, CYCLIC } kind = CONST;
    int64_t c = 0;  // CONST value
    int d = 0;      // launch dim
    int64_t s = 1;  // IPMUL factor; BLOCK / CYCLIC size
};

struct MSpace {
    std::vector<tm_op> ops;
    std::vector<int64_t> shape;
};

struct Value {
    enum Kind { SCALAR, TUPLE, MACHINE, TASK } kind = SCALAR;
    Scalar sc;
    std::vector<Scalar> tup;
    MSpace ms;
};

struct Context {
    int lrank = 0;
    int64_t extent[TM_MAX_LRANK] = {0, 0, 0, 0};
    int32_t nodes = 0, gpus = 0;
    int32_t halo[TM_MAX_LRANK] = {1, 1, 1, 1};
};

Value constant(int64_t c) {
    Value v;
    v.sc.c = c;
    return v;
}

bool is_const(const Scalar& s) { return s.kind == Scalar::CONST; }

// floor division / modulo of non-negative operands (reading of the paper's
// integer arithmetic); negative results are not produced by mappers.
Scalar arith(const Tok& at, char op, const Scalar& a, const Scalar& b, const Context& cx) {
    Scalar r;
    if (is_const(a) && is_const(b)) {
        switch (op) {
            case '+': r.c = a.c + b.c; break;
            case '-': r.c = a.c - b.c; break;
            case '*': r.c = a.c * b.c; break;
            case '/':
                if (b.c <= 0 || a.c < 0) fail(at, "division needs a non-negative dividend and a positive divisor");
                r.c = a.c / b.c;
                break;
            case '%':
                if (b.c <= 0 || a.c < 0) fail(at, "modulo needs a non-negative dividend and a positive divisor");
                r.c = a.c % b.c;
                break;
        }
        return r;
    }
    if (op == '*' && a.kind == Scalar::IP && is_const(b) && b.c >= 1) return Scalar{Scalar::IPMUL, 0, a.d, b.c};
    if (op == '*' && b.kind == Scalar::IP && is_const(a) && a.c >= 1) return Scalar{Scalar::IPMUL, 0, b.d, a.c};
    if (op == '/' && a.kind == Scalar::IPMUL && is_const(b)) {
        if (b.c != cx.extent[a.d])
            fail(at, "an index-point term ip[d]*s must be divided by the launch extent of dim d (block projection)");
        return Scalar{Scalar::BLOCK, 0, a.d, a.s};
    }
    if (op == '%' && a.kind == Scalar::IP && is_const(b) && b.c >= 1) return Scalar{Scalar::CYCLIC, 0, a.d, b.c};
    fail(at, "unsupported arithmetic on the index point (only ip[d]*s/ispace[d] and ip[d]%s are projections)");
}

Value arith(const Tok& at, char op, const Value& a, const Value& b, const Context& cx) {
    auto scalars = [&](const Value& v) -> const std::vector<Scalar>* {
        return v.kind == Value::TUPLE ? &v.tup : nullptr;
    };
    if ((a.kind != Value::SCALAR && a.kind != Value::TUPLE) || (b.kind != Value::SCALAR && b.kind != Value::TUPLE))
        fail(at, "arithmetic needs integers or tuples");
    const auto* ta = scalars(a);
    const auto* tb = scalars(b);
    if (!ta && !tb) {
        Value r;
        r.sc = arith(at, op, a.sc, b.sc, cx);
        return r;
    }
    Value r;
    r.kind = Value::TUPLE;
    const size_t n = ta ? ta->size() : tb->size();
    if (ta && tb && ta->size() != tb->size()) fail(at, "tuple sizes differ");
    for (size_t i = 0; i < n; ++i) r.tup.push_back(arith(at, op, ta ? (*ta)[i] : a.sc, tb ? (*tb)[i] : b.sc, cx));
    return r;
}

int64_t as_int(const Tok& at, const Value& v, const char* what) {
    if (v.kind != Value::SCALAR || !is_const(v.sc)) fail(at, std::string(what) + " must be an integer constant");
    return v.sc.c;
}

std::vector<int64_t> as_ints(const Tok& at, const Value& v, const char* what) {
    std::vector<int64_t> out;
    if (v.kind == Value::SCALAR) {
        out.push_back(as_int(at, v, what));
        return out;
    }
    if (v.kind != Value::TUPLE) fail(at, std::string(what) + " must be a tuple of integers");
    for (const auto& s : v.tup) {
        if (!is_const(s)) fail(at, std::string(what) + " must be a tuple of integers");
        out.push_back(s.c);
    }
    return out;
}

Value sizes_of(const MSpace& m) {
    Value v;
    v.kind = Value::TUPLE;
    for (int64_t s : m.shape) v.tup.push_back(Scalar{Scalar::CONST, s, 0, 1});
    return v;
}

// Processor-space methods (Fig. 6, Sec. 4.2): record the op and the new shape.
MSpace apply(const Tok& at, const MSpace& m, const std::string& name, const std::vector<Value>& args,
             const Context& cx) {
    MSpace r = m;
    const int rank = (int)m.shape.size();
    if ((int)r.ops.size() >= TM_MAX_OPS) fail(at, "more than 8 transformations");
    tm_op op{};
    auto dim = [&](const Value& v, const char* what) {
        const int64_t i = as_int(at, v, what);
        if (i < 0 || i >= rank) fail(at, std::string(what) + " out of range");
        return (int)i;
    };
    if (name == "split" || name == "balance_split") {
        if (args.size() != 2) fail(at, name + " takes (dim, factor)");
        const int i = dim(args[0], "dim");
        const int64_t d = as_int(at, args[1], "factor");
        if (d < 1) fail(at, "factor must be positive");
        if (name == "split" && m.shape[i] % d) fail(at, "split factor must divide the dim");
        op.kind = name == "split" ? TM_SPLIT : TM_BALANCE_SPLIT;
        op.a = i;
        op.b = (int32_t)d;
        const int64_t rest = name == "split" ? m.shape[i] / d : (m.shape[i] + d - 1) / d;
        r.shape.erase(r.shape.begin() + i);
        r.shape.insert(r.shape.begin() + i, {d, rest});
    } else if (name == "merge") {
        if (args.size() != 2) fail(at, "merge takes (p, q)");
        const int p = dim(args[0], "p"), q = dim(args[1], "q");
        if (p >= q) fail(at, "merge needs p < q");
        op.kind = TM_MERGE;
        op.a = p;
        op.b = q;
        r.shape[p] = m.shape[p] * m.shape[q];
        r.shape.erase(r.shape.begin() + q);
    } else if (name == "swap") {
        if (args.size() != 2) fail(at, "swap takes (p, q)");
        const int p = dim(args[0], "p"), q = dim(args[1], "q");
        if (p == q) fail(at, "swap needs p != q");
        op.kind = TM_SWAP;
        op.a = p;
        op.b = q;
        std::swap(r.shape[p], r.shape[q]);
    } else if (name == "decompose") {
        if (args.size() != 2) fail(at, "decompose takes (dim, domain)");
        const int i = dim(args[0], "dim");
        const std::vector<int64_t> dom = as_ints(at, args[1], "domain");
        const int k = (int)dom.size();
        if (k < 1 || k > TM_MAX_LRANK) fail(at, "decompose over 1..4 dims");
        int64_t ext[TM_MAX_LRANK];
        int32_t h[TM_MAX_LRANK], f[TM_MAX_LRANK];
        for (int a = 0; a < k; ++a) {
            if (dom[a] < 1) fail(at, "decompose domain sizes must be positive");
            ext[a] = dom[a];
            h[a] = k == cx.lrank ? cx.halo[a] : 1;
        }
        if (tm_decompose_argmin(m.shape[i], k, ext, h, f) != TM_OK) fail(at, std::string("decompose: ") + tm_last_error());
        op.kind = TM_DECOMPOSE;
        op.a = i;
        op.nf = k;
        for (int a = 0; a < k; ++a) op.f[a] = f[a];
        r.shape.erase(r.shape.begin() + i);
        r.shape.insert(r.shape.begin() + i, f, f + k);
    } else {
        fail(at, "unknown processor-space method '" + name + "'");
    }
    if ((int)r.shape.size() > TM_MAX_MRANK) fail(at, "processor space of rank above 8");
    r.ops.push_back(op);
    return r;
}

// ------------------------------------------------------------------ parser / evaluator

struct Function {
    std::vector<std::string> params;
    std::vector<std::string> types;
    std::vector<const Line*> body;
};

struct Result {
    bool done = false;
    MSpace ms;
    std::vector<Scalar> coords;
};

class Eval {
   public:
    Eval(const Context& cx, std::map<std::string, Value>& env) : cx_(cx), env_(env) {}

    Value expr(const std::vector<Tok>& t, size_t& i) { return additive(t, i); }

    // Index list `[a, *b, ...]` or a slice `[x:y]` after `[` has been consumed.
    void index(const std::vector<Tok>& t, size_t& i, const Value& base, Value& out, bool& is_selection,
               std::vector<Scalar>& sel) {
        const Tok& at = t[i - 1];
        // slice?
        size_t j = i;
        int depth = 0;
        bool colon = false;
        for (; j < t.size(); ++j) {
            if (t[j].text == "[" || t[j].text == "(") ++depth;
            if (t[j].text == "]" || t[j].text == ")") {
                if (depth == 0) break;
                --depth;
            }
            if (depth == 0 && t[j].text == ":") colon = true;
        }
        if (j >= t.size()) fail(at, "unclosed '['");
        if (colon) {
            std::vector<Scalar> items = base.kind == Value::MACHINE ? sizes_of(base.ms).tup : base.tup;
            if (base.kind != Value::MACHINE && base.kind != Value::TUPLE) fail(at, "only tuples can be sliced");
            const int64_t n = (int64_t)items.size();
            int64_t lo = 0, hi = n;
            if (t[i].text != ":") lo = as_int(t[i], expr(t, i), "slice bound");
            expect(t, i, ":");
            if (t[i].text != "]") hi = as_int(t[i], expr(t, i), "slice bound");
            expect(t, i, "]");
            if (lo < 0) lo += n;
            if (hi < 0) hi += n;
            lo = std::max<int64_t>(0, std::min(lo, n));
            hi = std::max<int64_t>(lo, std::min(hi, n));
            out = Value{};
            out.kind = Value::TUPLE;
            out.tup.assign(items.begin() + lo, items.begin() + hi);
            is_selection = false;
            return;
        }
        std::vector<Scalar> items;
        bool unpacked = false;
        while (t[i].text != "]") {
            if (t[i].text == "*") {
                ++i;
                Value v = postfix(t, i);
                if (v.kind == Value::MACHINE) v = sizes_of(v.ms);
                if (v.kind != Value::TUPLE) fail(t[i - 1], "only tuples can be unpacked");
                items.insert(items.end(), v.tup.begin(), v.tup.end());
                unpacked = true;
            } else {
                Value v = expr(t, i);
                if (v.kind != Value::SCALAR) fail(t[i - 1], "index items must be integers");
                items.push_back(v.sc);
            }
            if (t[i].text == ",") ++i;
            else if (t[i].text != "]") fail(t[i], "expected ',' or ']'");
        }
        ++i;
        if (base.kind == Value::MACHINE && (unpacked || items.size() > 1 || !is_const(items[0]))) {
            is_selection = true;  // m[...] selects a processor
            sel = items;
            return;
        }
        if (items.size() != 1 || !is_const(items[0])) fail(at, "an index must be one integer");
        std::vector<Scalar> seq = base.kind == Value::MACHINE ? sizes_of(base.ms).tup : base.tup;
        if (base.kind != Value::MACHINE && base.kind != Value::TUPLE) fail(at, "only tuples can be indexed");
        int64_t k = items[0].c;
        if (k < 0) k += (int64_t)seq.size();
        if (k < 0 || k >= (int64_t)seq.size()) fail(at, "index out of range");
        out = Value{};
        out.sc = seq[(size_t)k];  // an integer index into a processor space means its size (App. A.1)
        is_selection = false;
    }

    Value postfix(const std::vector<Tok>& t, size_t& i) {
        Value v = primary(t, i);
        for (;;) {
            if (i < t.size() && t[i].text == ".") {
                const Tok& at = t[++i];
                if (at.kind != T_NAME) fail(at, "expected a name after '.'");
                ++i;
                const std::string name = at.text;
                if (i < t.size() && t[i].text == "(") {
                    ++i;
                    std::vector<Value> args = call_args(t, i);
                    if (v.kind != Value::MACHINE) fail(at, "methods apply to processor spaces");
                    MSpace m = apply(at, v.ms, name, args, cx_);
                    v = Value{};
                    v.kind = Value::MACHINE;
                    v.ms = m;
                } else if (name == "size") {
                    if (v.kind != Value::MACHINE) fail(at, ".size applies to processor spaces");
                    v = sizes_of(v.ms);
                } else if (name == "ipoint" || name == "ispace") {
                    if (v.kind != Value::TASK) fail(at, "." + name + " applies to the task");
                    v = name == "ipoint" ? ipoint() : ispace();
                } else {
                    fail(at, "unknown attribute '" + name + "'");
                }
            } else if (i < t.size() && t[i].text == "[") {
                ++i;
                Value out;
                bool selection = false;
                std::vector<Scalar> sel;
                const Value base = v;
                index(t, i, base, out, selection, sel);
                if (selection) {
                    if (!returning_) fail(t[i - 1], "a processor can only be selected in a return statement");
                    result_.done = true;
                    result_.ms = base.ms;
                    result_.coords = sel;
                    return Value{};
                }
                v = out;
            } else {
                return v;
            }
        }
    }

    std::vector<Value> call_args(const std::vector<Tok>& t, size_t& i) {
        std::vector<Value> args;
        while (t[i].text != ")") {
            args.push_back(expr(t, i));
            if (t[i].text == ",") ++i;
            else if (t[i].text != ")") fail(t[i], "expected ',' or ')'");
        }
        ++i;
        return args;
    }

    Value primary(const std::vector<Tok>& t, size_t& i) {
        const Tok& at = t[i];
        if (at.kind == T_END) fail(at, "unexpected end of line");
        if (at.kind == T_INT) {
            ++i;
            return constant(at.value);
        }
        if (at.text == "-") {
            ++i;
            Value v = postfix(t, i);
            return arith(at, '-', constant(0), v, cx_);
        }
        if (at.text == "(") {
            ++i;
            std::vector<Value> items;
            bool tuple = false;
            while (t[i].text != ")") {
                if (t[i].text == "*") {
                    ++i;
                    Value v = postfix(t, i);
                    if (v.kind == Value::MACHINE) v = sizes_of(v.ms);
                    if (v.kind != Value::TUPLE) fail(t[i - 1], "only tuples can be unpacked");
                    for (const auto& s : v.tup) {
                        Value e;
                        e.sc = s;
                        items.push_back(e);
                    }
                    tuple = true;
                } else {
                    items.push_back(expr(t, i));
                }
                if (t[i].text == ",") {
                    tuple = true;
                    ++i;
                } else if (t[i].text != ")") {
                    fail(t[i], "expected ',' or ')'");
                }
            }
            ++i;
            if (!tuple && items.size() == 1) return items[0];
            Value v;
            v.kind = Value::TUPLE;
            for (const auto& e : items) {
                if (e.kind != Value::SCALAR) fail(at, "tuples hold integers");
                v.tup.push_back(e.sc);
            }
            return v;
        }
        if (at.kind == T_NAME) {
            ++i;
            if (at.text == "Machine") {
                expect(t, i, "(");
                const Tok& p = t[i];
                if (p.text != "GPU") fail(p, "only Machine(GPU) is modelled");
                ++i;
                expect(t, i, ")");
                Value v;
                v.kind = Value::MACHINE;
                v.ms.shape = {cx_.nodes, cx_.gpus};
                return v;
            }
            auto it = env_.find(at.text);
            if (it == env_.end()) fail(at, "unknown name '" + at.text + "'");
            return it->second;
        }
        fail(at, "unexpected '" + at.text + "'");
    }

    Value multiplicative(const std::vector<Tok>& t, size_t& i) {
        Value v = postfix(t, i);
        while (i < t.size() && (t[i].text == "*" || t[i].text == "/" || t[i].text == "%" || t[i].text == "//")) {
            const Tok& at = t[i++];
            const Value r = postfix(t, i);
            v = arith(at, at.text == "//" ? '/' : at.text[0], v, r, cx_);
        }
        return v;
    }

    Value additive(const std::vector<Tok>& t, size_t& i) {
        Value v = multiplicative(t, i);
        while (i < t.size() && (t[i].text == "+" || t[i].text == "-")) {
            const Tok& at = t[i++];
            const Value r = multiplicative(t, i);
            v = arith(at, at.text[0], v, r, cx_);
        }
        return v;
    }

    static void expect(const std::vector<Tok>& t, size_t& i, const char* s) {
        if (t[i].text != s) fail(t[i], std::string("expected '") + s + "'");
        ++i;
    }

    Value ipoint() const {
        Value v;
        v.kind = Value::TUPLE;
        for (int d = 0; d < cx_.lrank; ++d) v.tup.push_back(Scalar{Scalar::IP, 0, d, 1});
        return v;
    }
    Value ispace() const {
        Value v;
        v.kind = Value::TUPLE;
        for (int d = 0; d < cx_.lrank; ++d) v.tup.push_back(Scalar{Scalar::CONST, cx_.extent[d], 0, 1});
        return v;
    }

    bool returning_ = false;
    Result result_;

   private:
    const Context& cx_;
    std::map<std::string, Value>& env_;
};

std::vector<Tok> with_end(const Line& l) {
    std::vector<Tok> t = l.toks;
    Tok e;
    e.kind = T_END;
    e.line = l.number;
    e.col = l.toks.empty() ? 1 : l.toks.back().col + (int)l.toks.back().text.size();
    t.push_back(e);
    return t;
}

// Runs a function body; returns the selected processor space and coordinates.
Result run(const Function& f, const Context& cx, std::map<std::string, Value> env) {
    // parameters: a Task, or (point, space) tuples
    Eval probe(cx, env);
    if (f.params.size() == 1) {
        Value task;
        task.kind = Value::TASK;
        env[f.params[0]] = task;
    } else if (f.params.size() == 2) {
        env[f.params[0]] = probe.ipoint();
        env[f.params[1]] = probe.ispace();
    } else {
        throw FrontError{f.body.empty() ? 0 : f.body[0]->number, 1,
                         "a mapping function takes (Task t) or (Tuple point, Tuple space)"};
    }
    for (const Line* l : f.body) {
        std::vector<Tok> t = with_end(*l);
        Eval ev(cx, env);
        size_t i = 0;
        if (t[0].kind == T_NAME && t[0].text == "return") {
            i = 1;
            ev.returning_ = true;
            ev.expr(t, i);
            if (!ev.result_.done) fail(t[0], "the mapper must return a processor, m[...]");
            if (t[i].kind != T_END) fail(t[i], "unexpected text after the return value");
            return ev.result_;
        }
        if (t.size() >= 3 && t[0].kind == T_NAME && t[1].text == "=") {
            i = 2;
            Value v = ev.expr(t, i);
            if (t[i].kind != T_END) fail(t[i], "unexpected text after the expression");
            env[t[0].text] = v;
            continue;
        }
        fail(t[0], "expected 'name = expression' or 'return ...'");
    }
    throw FrontError{f.body.empty() ? 0 : f.body.back()->number, 1, "the mapper has no return statement"};
}

void translate(const char* src, const char* task, const Context& cx, tm_candidate* out) {
    const std::vector<Line> lines = tokenize(src);
    std::map<std::string, Function> funcs;
    std::map<std::string, Value> globals;
    std::string mapper;
    for (size_t li = 0; li < lines.size(); ++li) {
        const Line& l = lines[li];
        if (l.indent > 0) fail(l.toks[0], "unexpected indentation");
        const std::vector<Tok> t = with_end(l);
        if (t[0].text == "def") {
            if (t[1].kind != T_NAME || t[2].text != "(") fail(t[0], "expected 'def name(...):'");
            Function f;
            size_t i = 3;
            while (t[i].text != ")") {
                std::vector<std::string> words;
                while (t[i].kind == T_NAME) words.push_back(t[i++].text);
                if (words.empty() || words.size() > 2) fail(t[i], "expected '[Type] name'");
                f.params.push_back(words.back());
                f.types.push_back(words.size() == 2 ? words[0] : "");
                if (t[i].text == ",") ++i;
                else if (t[i].text != ")") fail(t[i], "expected ',' or ')'");
            }
            ++i;
            if (t[i].text != ":") fail(t[i], "expected ':'");
            while (li + 1 < lines.size() && lines[li + 1].indent > 0) f.body.push_back(&lines[++li]);
            funcs[t[1].text] = f;
        } else if (t[0].text == "IndexTaskMap") {
            if (t[1].kind != T_NAME && t[1].text != "*") fail(t[1], "expected a task name");
            if (t[2].kind != T_NAME) fail(t[2], "expected a function name");
            if (t[1].text == task || (t[1].text == "*" && mapper.empty())) mapper = t[2].text;
        } else if (t.size() >= 3 && t[0].kind == T_NAME && t[1].text == "=") {
            Eval ev(cx, globals);
            size_t i = 2;
            Value v = ev.expr(t, i);
            if (t[i].kind != T_END) fail(t[i], "unexpected text after the expression");
            globals[t[0].text] = v;
        }
        // other statements (task, region, layout, collection and backpressure
        // directives) do not affect index mapping
    }
    if (mapper.empty()) throw FrontError{0, 0, std::string("no IndexTaskMap for task '") + task + "'"};
    auto fit = funcs.find(mapper);
    if (fit == funcs.end()) throw FrontError{0, 0, "IndexTaskMap names an undefined function '" + mapper + "'"};
    const Result r = run(fit->second, cx, globals);

    // processor coordinates -> projections
    const MSpace& m = r.ms;
    const Tok at = fit->second.body.empty() ? Tok{} : fit->second.body.back()->toks[0];
    if (r.coords.size() != m.shape.size())
        fail(at, "the processor index has " + std::to_string(r.coords.size()) + " coordinates for a space of rank " +
                     std::to_string(m.shape.size()));
    std::memset(out, 0, sizeof(*out));
    out->lrank = cx.lrank;
    out->nodes = cx.nodes;
    out->gpus_per_node = cx.gpus;
    for (int d = 0; d < cx.lrank; ++d) out->extent[d] = cx.extent[d];
    out->nops = (int32_t)m.ops.size();
    for (size_t t = 0; t < m.ops.size(); ++t) out->ops[t] = m.ops[t];
    out->mrank = (int32_t)m.shape.size();
    for (size_t j = 0; j < r.coords.size(); ++j) {
        const Scalar& s = r.coords[j];
        if (s.kind == Scalar::BLOCK && s.s == m.shape[j]) {
            out->proj_src[j] = (int8_t)s.d;
            out->proj_mode[j] = TM_BLOCK;
        } else if (s.kind == Scalar::CYCLIC && s.s == m.shape[j]) {
            out->proj_src[j] = (int8_t)s.d;
            out->proj_mode[j] = TM_CYCLIC;
        } else if (s.kind == Scalar::CONST && s.c == 0 && m.shape[j] == 1) {
            out->proj_src[j] = 0;  // a dim of size 1: every projection gives 0
            out->proj_mode[j] = TM_BLOCK;
        } else {
            fail(at, "processor coordinate " + std::to_string(j) +
                         " is not ip[d]*s/ispace[d] or ip[d]%s with s the size of that processor dim");
        }
    }
}

}  // namespace

extern "C" int tm_parse_index_task_map(const char* source, const char* task, int32_t lrank, const int64_t* extent,
                                       int32_t nodes, int32_t gpus_per_node, const int32_t* halo, tm_candidate* out) {
    if (!source || !task || !extent || !out) return tmk::set_error(TM_EINVAL, "null argument");
    if (lrank < 1 || lrank > TM_MAX_LRANK) return tmk::set_error(TM_EINVAL, "lrank %d", lrank);
    if (nodes < 1 || gpus_per_node < 1 || (int64_t)nodes * gpus_per_node > TM_MAX_VOLUME)
        return tmk::set_error(TM_EINVAL, "machine %d x %d", nodes, gpus_per_node);
    Context cx;
    cx.lrank = lrank;
    cx.nodes = nodes;
    cx.gpus = gpus_per_node;
    for (int d = 0; d < lrank; ++d) {
        if (extent[d] < 1 || extent[d] > TM_MAX_EXTENT) return tmk::set_error(TM_EINVAL, "extent[%d]", d);
        cx.extent[d] = extent[d];
        if (halo) {
            if (halo[d] < 0 || halo[d] > TM_MAX_HALO) return tmk::set_error(TM_EINVAL, "halo[%d]", d);
            cx.halo[d] = halo[d];
        }
    }
    try {
        translate(source, task, cx, out);
    } catch (const FrontError& e) {
        return tmk::set_error(TM_EINVAL, "line %d, column %d: %s", e.line, e.col, e.msg.c_str());
    } catch (const std::exception& e) {
        return tmk::set_error(TM_ENOMEM, "%s", e.what());
    }
    tmk::Shapes sh;
    const int rc = tmk::validate_shapes(out, &sh);
    if (rc != TM_OK) return tmk::set_error(rc, "translated mapper: %s", tm_last_error());
    return TM_OK;
}
