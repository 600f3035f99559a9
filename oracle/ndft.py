"""Direct (non-fast) trigonometric sums of NFFT fast summation, FP64.

Test infrastructure only (see ``oracle/__init__.py``).

Fast summation (Section 3.1, eq. (fastsum)) replaces the kernel by an
h-periodic trigonometric polynomial with coefficients b_k on the index set
I_N = {-N/2, ..., N/2-1}^d (eq. (ansatz_NFFT)) and evaluates

    t_i = sum_k b_k ( sum_j w_j exp(-2 pi i k.y_j / h) ) exp(2 pi i k.x_i / h).

Here the sums are done literally: the inner sum is ``ndft_adjoint``, the outer
sum ``ndft_trafo``.  Points are given in units of the period (h = 1), i.e. on
the torus [-1/2, 1/2)^d.  The kernel sum of a real kernel is real; the value
returned by ``fastsum_ndft`` is the real part of the complex sum over I_N.
"""
import itertools

import numpy as np


def _points(a):
    """Point array of shape (n, d); a 1-D array is n points in one dimension."""
    a = np.asarray(a, dtype=np.float64)
    return a[:, None] if a.ndim == 1 else a


def index_set(N, d):
    """All k in I_N = {-N/2, ..., N/2-1}^d, shape (N**d, d), last index fastest."""
    if N % 2:
        raise ValueError("N must be even (N in 2N)")
    one = np.arange(-N // 2, N // 2)
    grids = np.meshgrid(*([one] * d), indexing="ij")
    return np.stack([g.ravel() for g in grids], axis=-1).astype(np.float64)


def ndft_adjoint(y, w, N):
    """fhat_k = sum_j w_j exp(-2 pi i k.y_j) for k in I_N (inner sum of eq. (fastsum)).

    Returns an array of shape (N,)*d indexed by k + N/2.
    """
    y = _points(y)
    d = y.shape[1]
    k = index_set(N, d)
    ph = np.exp(-2j * np.pi * (k @ y.T))          # (N^d, n)
    return (ph @ np.asarray(w, dtype=np.complex128)).reshape((N,) * d)


def ndft_trafo(fhat, x, N):
    """f_i = sum_k fhat_k exp(2 pi i k.x_i) for k in I_N (outer sum of eq. (fastsum))."""
    x = _points(x)
    d = fhat.ndim
    k = index_set(N, d)
    ph = np.exp(2j * np.pi * (x @ k.T))            # (n, N^d)
    return ph @ np.asarray(fhat, dtype=np.complex128).ravel()


def gauss_coeffs(N, d, eps_t):
    """Fourier coefficients on I_N of the 1-periodized kernel exp(-|z|^2/eps_t).

    For period 1, the k-th Fourier coefficient of sum_l K(z + l) equals the
    continuous Fourier transform of K at k (Poisson summation), which for the
    Gaussian is (pi eps_t)^(d/2) exp(-pi^2 eps_t |k|^2).  These are the b_k of
    eq. (ansatz_NFFT) when the Gaussian is regularized by periodization.
    """
    k = index_set(N, d)
    k2 = np.sum(k * k, axis=1)
    return ((np.pi * eps_t) ** (d / 2.0) * np.exp(-np.pi ** 2 * eps_t * k2)).reshape((N,) * d)


def periodized_gauss(z, eps_t, images=4):
    """sum over l in {-images..images}^d of exp(-|z + l|^2/eps_t), by brute force."""
    z = _points(z)
    d = z.shape[1]
    out = np.zeros(z.shape[0])
    for l in itertools.product(range(-images, images + 1), repeat=d):
        zz = z + np.asarray(l, dtype=np.float64)
        out += np.exp(-np.sum(zz * zz, axis=1) / eps_t)
    return out


def fastsum_ndft(x, y, w, b):
    """Re of eq. (fastsum) with given coefficients b (shape (N,)*d)."""
    N = b.shape[0]
    return np.real(ndft_trafo(b * ndft_adjoint(y, w, N), x, N))
