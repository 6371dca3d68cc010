"""ctypes signatures of the ranker entry points (filled in by the ranker module)."""


def declare(L):
    return L
