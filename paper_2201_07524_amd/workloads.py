"""Seeded synthetic point clouds shaped like the paper's workloads.

This module only draws random inputs; it holds none of the method's
arithmetic and is shared by the tests, the benchmark and the oracle checks.
Every generator uses numpy's PCG64 ``default_rng(seed)`` and returns float64
arrays: points of shape (n, d) and probability vectors of shape (n,).

Workloads (the paper's data sets are replaced by these stand-ins):
  * ``plain_1d``     d = 1, i.i.d. uniform on [-1/4, 1/4], uniform weights
                     (the one-dimensional synthetic experiment of Section 4.1.1).
  * ``gmm_2d``       d = 2, 5-component isotropic Gaussian mixtures (sigma 0.03,
                     means uniform in [-0.2, 0.2]^2), Dirichlet(1) weights.
  * ``ball_shell_3d`` d = 3, uniform in a ball of radius 0.2 against a noisy
                     sphere shell (radius 0.15, noise 0.01), uniform weights.
  * ``batched_2d``   many independent d = 2 mixture problems with log-uniform
                     sizes and per-problem temperature.
  * ``gmm_3d``       d = 3 mixtures for the differentiated form.
  * ``uniform_square`` uniform on [0,1]^2 (the two-dimensional experiment of
                     Section 4.1.2).
  * ``pixel_grid_pair`` two k x k images on one pixel grid in [0,1]^2 with
                     smoothed Gaussian random-field intensities: the shape of
                     the benchmark-image experiments of Section 4.2 (32^2 to
                     512^2 pixels).  It is not that data set's images.
"""
import numpy as np


def uniform_weights(n):
    return np.full(n, 1.0 / n)


def dirichlet_weights(n, seed):
    """Dirichlet(1, ..., 1): normalized i.i.d. standard exponentials."""
    e = np.random.default_rng(seed).standard_exponential(n)
    return e / e.sum()


def gaussian_mixture(n, d, seed, components=5, sigma=0.03, box=0.2):
    """n points from an equal-weight isotropic mixture; means uniform in [-box, box]^d."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-box, box, size=(components, d))
    labels = rng.integers(0, components, size=n)
    return means[labels] + sigma * rng.standard_normal((n, d))


def uniform_ball(n, seed, radius=0.2, d=3):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((n, d))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    rad = radius * rng.uniform(0.0, 1.0, size=n) ** (1.0 / d)
    return u * rad[:, None]


def noisy_shell(n, seed, radius=0.15, noise=0.01, d=3):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((n, d))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    rad = radius + noise * rng.standard_normal(n)
    return u * rad[:, None]


def plain_1d(n=2048):
    """Plain 1-D problem: n = 2048 by default, eps = 0.05, r = 2."""
    rng_x = np.random.default_rng(101)
    rng_y = np.random.default_rng(102)
    x = rng_x.uniform(-0.25, 0.25, size=(n, 1))
    y = rng_y.uniform(-0.25, 0.25, size=(n, 1))
    return dict(x=x, p=uniform_weights(n), y=y, pt=uniform_weights(n), d=1, r=2, eps=0.05,
                N=256, m=8, sigma=2.0, iters=200, precision="fp64")


def gmm_2d(n=1_000_000):
    """2-D mixtures at scale: n = 1e6 by default, eps = 0.01, r = 2, N = 512."""
    x = gaussian_mixture(n, 2, 201)
    y = gaussian_mixture(n, 2, 202)
    return dict(x=x, p=dirichlet_weights(n, 203), y=y, pt=dirichlet_weights(n, 204), d=2, r=2,
                eps=0.01, N=512, m=8, sigma=2.0, iters=500, precision="fp32")


def ball_shell_3d(n=4_000_000):
    """3-D ball against shell: n = 4e6 by default, eps = 0.02, Euclidean cost r = 1."""
    x = uniform_ball(n, 301)
    y = noisy_shell(n, 302)
    return dict(x=x, p=uniform_weights(n), y=y, pt=uniform_weights(n), d=3, r=1, eps=0.02,
                N=128, m=6, sigma=2.0, iters=300, precision="fp32")


def gmm_3d(n=1_000_000):
    """3-D mixtures for the differentiated form: eps = 0.01, r = 2, N = 128, m = 8."""
    x = gaussian_mixture(n, 3, 501)
    y = gaussian_mixture(n, 3, 502)
    return dict(x=x, p=uniform_weights(n), y=y, pt=uniform_weights(n), d=3, r=2, eps=0.01,
                N=128, m=8, sigma=2.0, iters=300, precision="fp32")


def batched_sizes(B=512, seed=400, lo=1e3, hi=2e5):
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=B))).astype(np.int64)
    eps = rng.uniform(0.005, 0.05, size=B)
    return sizes, eps


def batched_2d(B=512, seed=400, lo=1e3, hi=2e5):
    """B independent 2-D mixture problems with log-uniform sizes n_b in [lo, hi].

    Returns a list of dicts (x, p, y, pt, eps) plus the shared parameters.
    """
    sizes, eps = batched_sizes(B, seed, lo, hi)
    probs = []
    for b in range(B):
        n = int(sizes[b])
        x = gaussian_mixture(n, 2, 400000 + 2 * b)
        y = gaussian_mixture(n, 2, 400000 + 2 * b + 1)
        probs.append(dict(x=x, p=uniform_weights(n), y=y, pt=uniform_weights(n), eps=float(eps[b])))
    return dict(problems=probs, d=2, r=2, N=256, m=6, sigma=2.0, iters=300, precision="fp32")


def uniform_square(n, seed=600):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(n, 2))
    y = rng.uniform(0.0, 1.0, size=(n, 2))
    return dict(x=x, p=uniform_weights(n), y=y, pt=uniform_weights(n), d=2, r=2, eps=0.05)


def smoothed_field(k, seed, length=0.08):
    """Gaussian random field on a k x k periodic pixel grid: white noise
    filtered by a Gaussian of standard deviation ``length`` (in units of the
    unit square) through the FFT, then shifted by one standard deviation and
    clipped at zero (about one pixel in six is zero) and normalized to sum one."""
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((k, k))
    f = np.fft.fftfreq(k)
    filt = np.exp(-2.0 * (np.pi * length * k) ** 2 * (f[:, None] ** 2 + f[None, :] ** 2))
    field = np.real(np.fft.ifft2(np.fft.fft2(noise) * filt))
    field = (field - field.mean()) / field.std() + 1.0
    w = np.clip(field, 0.0, None).ravel()
    return w / w.sum()


def pixel_grid_pair(k, seed=800):
    """Two images on the same k x k grid of pixel centers ((i + 1/2)/k, (j + 1/2)/k),
    intensities from independent smoothed fields (seeds ``seed``, ``seed + 1``);
    eps = 0.05 (the paper's lambda = 20), squared Euclidean cost."""
    c = (np.arange(k) + 0.5) / k
    g = np.stack(np.meshgrid(c, c, indexing="ij"), axis=-1).reshape(-1, 2)
    return dict(x=g, p=smoothed_field(k, seed), y=g.copy(), pt=smoothed_field(k, seed + 1), d=2, r=2, eps=0.05)


def subsample(cfg, n, seed=7):
    """Random subsample of both clouds of a workload, weights renormalized to sum one."""
    rng = np.random.default_rng(seed)
    ix = np.sort(rng.choice(cfg["x"].shape[0], size=n, replace=False))
    iy = np.sort(rng.choice(cfg["y"].shape[0], size=n, replace=False))
    out = dict(cfg)
    out["x"] = cfg["x"][ix]
    out["y"] = cfg["y"][iy]
    out["p"] = cfg["p"][ix] / cfg["p"][ix].sum()
    out["pt"] = cfg["pt"][iy] / cfg["pt"][iy].sum()
    return out
