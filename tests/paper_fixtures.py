"""Loaders for the paper's printed integer examples (tests/golden/paper_examples.json)."""
import json
import os

import numpy as np

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_examples.json")


def examples():
    with open(_PATH) as f:
        return json.load(f)


def fold(mat, n, dims):
    """Inverse of the paper's mode-n unfolding: columns run over the remaining modes in
    increasing order, the earliest remaining mode fastest."""
    mat = np.asarray(mat, dtype=np.float64)
    dims = tuple(int(x) for x in dims)
    assert mat.shape == (dims[n], int(np.prod(dims)) // dims[n])
    rest = [k for k in range(len(dims)) if k != n]
    X = np.zeros(dims)
    for idx in np.ndindex(*dims):
        col, stride = 0, 1
        for k in rest:
            col += idx[k] * stride
            stride *= dims[k]
        X[idx] = mat[idx[n], col]
    return X


def fold_ex6(mat, dims):
    """Example 6's display: rows = mode-2 index, column = N3*i1 + i3."""
    mat = np.asarray(mat, dtype=np.float64)
    X = np.zeros(dims)
    for i, j, k in np.ndindex(*dims):
        X[i, j, k] = mat[j, dims[2] * i + k]
    return X


def arr(x):
    return np.asarray(x, dtype=np.float64)
