"""Helpers shared by the GPU tests (no solver arithmetic here)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def gpu_available():
    return torch.cuda.is_available()


def rel_err(X, Y):
    """Per-instance ||X - Y||_F / ||Y||_F over the last two axes."""
    num = np.sqrt(((X - Y) ** 2).sum(axis=(-1, -2)))
    den = np.sqrt((Y ** 2).sum(axis=(-1, -2)))
    return num / np.where(den == 0, 1.0, den)
