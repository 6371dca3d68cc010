"""ctypes signatures of the ranker and search entry points of libtaskmap."""
import ctypes

P, I32, I64, U64, F32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float

SIGNATURES = {
    "tm_ranker_param_count": [],
    "tm_ranker_feature_count": [],
    "tm_ranker_create": [U64, P],
    "tm_ranker_destroy": [P],
    "tm_ranker_get_params": [P, P, P],
    "tm_ranker_set_params": [P, P, P],
    "tm_ranker_get_scaling": [P, P],
    "tm_ranker_features": [P, P, P],
    "tm_ranker_block_estimates": [P, P, P],
    "tm_ranker_forward": [P, P, I64, P, P],
    "tm_ranker_grad": [P, P, P, I64, P, P],
    "tm_ranker_train": [P, P, P, I64, I32, I32, F32, U64, P, P],
    "tm_ranker_save": [P, ctypes.c_char_p],
    "tm_ranker_load": [ctypes.c_char_p, P],
    "tm_search": [P, P, P, I64, I32, I32, F32, F32, P, P, P],
}


def declare(L):
    for name, args in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = ctypes.c_int
        fn.argtypes = args
    return L
