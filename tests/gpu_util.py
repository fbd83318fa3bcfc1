"""Helpers shared by the GPU tests (no solver arithmetic here)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def gpu_available():
    return torch.cuda.is_available()


def frob_err(X, Y):
    """Per-instance ||X - Y||_F / ||Y||_F over the last two axes."""
    num = np.sqrt(((X - Y) ** 2).sum(axis=(-1, -2)))
    den = np.sqrt((Y ** 2).sum(axis=(-1, -2)))
    return num / np.where(den == 0, 1.0, den)


def elem_err(X, Y):
    """Per-instance max over entries of |x_ij - y_ij| / max_i |y_ij|: every
    entry against the largest entry of its own column (columns of zeros
    against 1)."""
    colmax = np.abs(Y).max(axis=-2, keepdims=True)
    return (np.abs(X - Y) / np.where(colmax == 0, 1.0, colmax)).max(axis=(-1, -2))


def rel_err(X, Y):
    """Per-instance error used by the parity bars: the larger of the
    normwise relative error and the entry-wise error against each column's
    largest entry, so that a bar holds for every entry as well as for the
    matrix."""
    return np.maximum(frob_err(X, Y), elem_err(X, Y))
