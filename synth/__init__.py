"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module only draws random numbers (numpy PCG64 streams keyed by a seed).
It holds none of the spectral-element arithmetic: no GLL points, no mesh
numbering, no geometry, no operator.  Whatever a caller needs to turn these
draws into method inputs (scattering a unique-node field to the local layout,
evaluating a Fourier sum at node coordinates) each side does with its own code.

Recipes (shapes and distributions of the paper's cubic-mesh workloads, Sec. 4.4,
widened to the solver workloads the library serves):
  * ``unique_normal``      u_G ~ N(0, 1) on the unique nodes of a periodic box.
  * ``unique_uniform``     h1_G ~ U[lo, hi] on the unique nodes.
  * ``local_normal``       element-local random fields, [E][lx][lx][lx].
  * ``random_spd_factors`` six symmetric-positive-definite geometric factors
                           per node plus a positive h1, for operator tests that
                           do not need a mesh.
  * ``fourier_modes``      32 modes: integer wave vectors k (||k||_inf <= kmax,
                           k != 0), amplitudes ~ N(0, 1), phases ~ U[0, 2 pi).
  * ``amplitudes``         deformation amplitudes ~ U[lo, hi].
"""
import numpy as np

__all__ = ["rng", "unique_normal", "unique_uniform", "local_normal",
           "random_spd_factors", "fourier_modes", "amplitudes"]


def rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def unique_normal(count, seed):
    """``count`` float64 draws from N(0, 1)."""
    return rng(seed).standard_normal(int(count))


def unique_uniform(count, lo, hi, seed):
    """``count`` float64 draws from U[lo, hi)."""
    return rng(seed).uniform(lo, hi, int(count))


def local_normal(nel, lx, seed):
    """float64 array of shape (nel, lx, lx, lx), entries ~ N(0, 1)."""
    return rng(seed).standard_normal((int(nel), lx, lx, lx))


def random_spd_factors(nel, lx, seed, h1_range=(0.5, 2.0)):
    """Six arrays (g11, g22, g33, g12, g13, g23) and h1, each (nel, lx, lx, lx).

    Per node the 3x3 matrix [[g11,g12,g13],[g12,g22,g23],[g13,g23,g33]] is
    symmetric positive definite: it is L L^T + 0.1 I for a random lower
    triangular L with N(0, 1) entries.  h1 ~ U[h1_range).
    """
    r = rng(seed)
    shp = (int(nel), lx, lx, lx)
    l11, l21, l22, l31, l32, l33 = (r.standard_normal(shp) for _ in range(6))
    g11 = l11 * l11 + 0.1
    g22 = l21 * l21 + l22 * l22 + 0.1
    g33 = l31 * l31 + l32 * l32 + l33 * l33 + 0.1
    g12 = l11 * l21
    g13 = l11 * l31
    g23 = l21 * l31 + l22 * l32
    h1 = r.uniform(h1_range[0], h1_range[1], shp)
    return (g11, g22, g33, g12, g13, g23), h1


def fourier_modes(seed, count=32, kmax=8):
    """Random Fourier modes for a periodic right-hand side.

    Returns (k, amp, phase): k int64 (count, 3) with every component in
    [-kmax, kmax] and k != 0; amp ~ N(0, 1); phase ~ U[0, 2 pi).
    """
    r = rng(seed)
    ks = []
    while len(ks) < count:
        k = r.integers(-kmax, kmax + 1, 3)
        if np.any(k != 0):
            ks.append(k)
    k = np.array(ks, dtype=np.int64)
    amp = r.standard_normal(count)
    phase = r.uniform(0.0, 2.0 * np.pi, count)
    return k, amp, phase


def amplitudes(seed, count, lo=0.0, hi=0.2):
    """``count`` deformation amplitudes ~ U[lo, hi)."""
    return rng(seed).uniform(lo, hi, int(count))


# --- learned preconditioner: random draws the training method makes ----------
MLP_SIZES = (518, 256, 256, 512)   # inputs (residual + 6 geometric features), hidden, hidden, outputs


def mlp_init(seed, sizes=MLP_SIZES):
    """He-normal initial weights and zero biases: for each layer a float64
    (fan_out, fan_in) matrix ~ N(0, 2 / fan_in) and a zero vector."""
    r = rng(seed)
    params = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        params.append(r.standard_normal((fo, fi)) * np.sqrt(2.0 / fi))
        params.append(np.zeros(fo))
    return params


def permutation(seed, n):
    """A random permutation of range(n) (minibatch order)."""
    return rng(seed).permutation(int(n))


def choice(seed, n, k):
    """k distinct indices from range(n)."""
    return rng(seed).choice(int(n), size=int(k), replace=False)


def snapshot_iterations(seed, count, kmax):
    """``count`` iteration numbers spread log-uniformly over [1, kmax]."""
    r = rng(seed)
    ks = np.unique(np.round(np.exp(r.uniform(0.0, np.log(kmax), count))).astype(np.int64))
    return np.clip(ks, 1, kmax)
