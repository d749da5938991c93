"""Naive separable DFT in FP64 (the transform used throughout the Appendix).

Convention: forward  X[n] = sum_j x[j] exp(-2 pi i n j / N)   (unnormalised),
            inverse  x[j] = (1/N) sum_n X[n] exp(+2 pi i n j / N).
The twiddle exp(-2 pi i (n j mod N)/N) takes its argument after exact integer
reduction, so each entry is the correctly reduced angle.  The 3-D transform
applies the 1-D matrix along the last three axes; leading axes are batch.
"""
import functools
import numpy as np


@functools.lru_cache(maxsize=None)
def dft_matrix(N, sign=-1):
    n = np.arange(N)
    k = np.outer(n, n) % N
    return np.exp(sign * 2j * np.pi * k / N)


def _along(x, W, axis):
    x = np.moveaxis(x, axis, -1)
    y = x @ W.T
    return np.moveaxis(y, -1, axis)


def fft3(x):
    """Unnormalised forward 3-D DFT over the last three axes."""
    x = np.asarray(x, dtype=complex)
    N = x.shape[-1]
    W = dft_matrix(N, -1)
    for ax in (-3, -2, -1):
        x = _along(x, W, ax)
    return x


def ifft3(X):
    """Inverse 3-D DFT over the last three axes, including the 1/N^3."""
    X = np.asarray(X, dtype=complex)
    N = X.shape[-1]
    W = dft_matrix(N, +1)
    for ax in (-3, -2, -1):
        X = _along(X, W, ax)
    return X / N ** 3
