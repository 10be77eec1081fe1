"""Seeded synthetic inputs for the matrix square root workloads.

This module only draws random matrices with the sizes, value distributions and
structure of the workloads; it performs none of the square-root method's
arithmetic.  It is shared by the tests, the benchmark and the smoke check.
Everything is float64/complex128 NumPy on the host, column-major when handed to
a device (all matrices built here are square, and the ones that are not
symmetric are built so that either memory order is a valid input: the root of
A^T is the transpose of the root of A).

Constructions (each returns the exact factors that define the input, so a test
can form the known root without running any solver):

* ``spd(n, kappa, seed)``: A = Q diag(lam) Q^T with Q Haar-orthogonal and lam
  log-uniform on [kappa^-1/2, kappa^1/2], both endpoints pinned so that the
  2-norm condition number is exactly kappa.
* ``spd_range(n, lo, hi, seed)``: same with eigenvalues log-uniform in [lo, hi]
  (endpoints pinned).
* ``nonsym_shifted(n, seed)``: A = 2 I + G / sqrt(n), G i.i.d. N(0, 1).
* ``hpd(n, kappa, seed)``: complex Hermitian A = U diag(lam) U^H, U
  Haar-unitary, lam as in ``spd``.
* ``complex_square(n, seed)``: B = Q (D + N) Q^H with Q Haar-unitary, D diagonal
  uniform in the disk |z - 2| < 1.5, N strictly upper triangular complex normal
  with standard deviation 0.1/sqrt(n); A = B B.
* ``hilbert(n, tau)``: H_n + tau I with (H_n)_ij = 1/(i + j - 1), 1-based.
* ``table1(set_id, seed)``: the test sets I-VII of the paper's Table 1 (the
  unspecified shift is stated at ``TABLE1``).
"""

from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def haar_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the
    signs of diag(R) folded into Q (Mezzadri's construction)."""
    z = rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def haar_unitary(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed unitary matrix from a complex Ginibre matrix."""
    z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    ph = d / np.where(np.abs(d) == 0, 1.0, np.abs(d))
    return q * ph[None, :]


def loguniform_eigs(n: int, lo: float, hi: float, rng: np.random.Generator) -> np.ndarray:
    """n values log-uniform on [lo, hi] with the two endpoints pinned."""
    if n == 1:
        return np.array([np.sqrt(lo * hi)])
    lam = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))
    lam[0] = lo
    lam[-1] = hi
    return np.sort(lam)


def spd_range(n: int, lo: float, hi: float, seed: int):
    """Returns (A, Q, lam) with A = Q diag(lam) Q^T symmetrised exactly."""
    rng = _rng(seed)
    q = haar_orthogonal(n, rng)
    lam = loguniform_eigs(n, lo, hi, rng)
    a = (q * lam[None, :]) @ q.T
    a = 0.5 * (a + a.T)
    return np.asfortranarray(a), q, lam


def spd(n: int, kappa: float, seed: int):
    """SPD matrix with 2-norm condition number kappa, eigenvalues log-uniform
    on [kappa^-1/2, kappa^1/2]."""
    s = np.sqrt(kappa)
    return spd_range(n, 1.0 / s, s, seed)


def hpd(n: int, kappa: float, seed: int):
    """Complex Hermitian positive definite A = U diag(lam) U^H with U
    Haar-unitary and lam log-uniform on [kappa^-1/2, kappa^1/2] (endpoints
    pinned), made exactly Hermitian as (A + A^H)/2.  Returns (A, U, lam)."""
    rng = _rng(seed)
    u = haar_unitary(n, rng)
    s = np.sqrt(kappa)
    lam = loguniform_eigs(n, 1.0 / s, s, rng)
    a = (u * lam[None, :]) @ u.conj().T
    a = 0.5 * (a + a.conj().T)
    return np.asfortranarray(a), u, lam


def nonsym_shifted(n: int, seed: int) -> np.ndarray:
    """A = 2 I + G / sqrt(n) with G i.i.d. standard normal."""
    rng = _rng(seed)
    g = rng.standard_normal((n, n))
    return np.asfortranarray(2.0 * np.eye(n) + g / np.sqrt(n))


def complex_square(n: int, seed: int):
    """Returns (A, B) with A = B B, B = Q (D + N) Q^H.  D is uniform in the disk
    |z - 2| < 1.5 (so arg z < 48.6 degrees and B is the principal root of A)
    and N is strictly upper triangular complex normal, E|N_ij|^2 = 0.01/n."""
    rng = _rng(seed)
    q = haar_unitary(n, rng)
    rad = 1.5 * np.sqrt(rng.uniform(size=n))
    ang = 2.0 * np.pi * rng.uniform(size=n)
    d = 2.0 + rad * np.exp(1j * ang)
    sd = 0.1 / np.sqrt(n)
    nn = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * (sd / np.sqrt(2.0))
    nn = np.triu(nn, 1)
    tri = np.diag(d) + nn
    b = q @ tri @ q.conj().T
    a = b @ b
    return np.asfortranarray(a), np.asfortranarray(b)


def hilbert(n: int, tau: float) -> np.ndarray:
    i = np.arange(1, n + 1, dtype=np.float64)
    h = 1.0 / (i[:, None] + i[None, :] - 1.0)
    return np.asfortranarray(h + tau * np.eye(n))


# The test sets of the paper's Table 1: (kind, entry law, n).  "Plus shift"
# is unspecified there; the shift used here is 1.1 times the asymptotic
# radius of the centred bulk (sigma sqrt(n) for i.i.d. nonsymmetric entries,
# 2 sigma sqrt(n) for symmetric ones) plus 1, so the bulk lies in Re z > 1.
TABLE1 = {
    "I": ("nonsym", "uniform", 2048),
    "II": ("nonsym", "normal", 2048),
    "III": ("nonsym", "uniform", 4096),
    "IV": ("nonsym", "normal", 4096),
    "V": ("sym", "uniform", 4096),
    "VI": ("sym", "normal", 4096),
    "VII": ("hilbert", None, 1024),
}


def table1(set_id: str, seed: int, n: int = None):
    """Matrix of test set `set_id` (Table 1).  Returns (A, shift).
    I-IV: A_ij i.i.d. U(0,1) or N(0,1) plus shift; V-VI: A_ij i.i.d. for
    i >= j, mirrored, plus shift; VII: H_n + 1e-6 I (shift 1e-6)."""
    kind, law, n0 = TABLE1[set_id]
    n = n0 if n is None else n
    if kind == "hilbert":
        return hilbert(n, 1e-6), 1e-6
    rng = _rng(seed)
    g = rng.uniform(size=(n, n)) if law == "uniform" else rng.standard_normal((n, n))
    sigma = np.sqrt(1.0 / 12.0) if law == "uniform" else 1.0
    if kind == "sym":
        low = np.tril(g)
        g = low + np.tril(low, -1).T
        shift = 2.2 * sigma * np.sqrt(n) + 1.0
    else:
        shift = 1.1 * sigma * np.sqrt(n) + 1.0
    return np.asfortranarray(g + shift * np.eye(n)), float(shift)


def gaussian(shape, seed: int) -> np.ndarray:
    """i.i.d. N(0, 1) array (used for upstream gradients and FD directions)."""
    return _rng(seed).standard_normal(shape)


def nonsym_kappa(n: int, kappa: float, seed: int) -> np.ndarray:
    """Nonsymmetric matrix whose difficulty tracks kappa: A = Q (L + N) Q^T with
    Q Haar-orthogonal, L = diag(lam), lam log-uniform on [kappa^-1/2, kappa^1/2]
    (endpoints pinned) and N strictly upper triangular with
    N_ij = nu_ij sqrt(lam_i lam_j), nu_ij ~ N(0, (0.1 / sqrt(n))^2)."""
    rng = _rng(seed)
    q = haar_orthogonal(n, rng)
    s = np.sqrt(kappa)
    lam = loguniform_eigs(n, 1.0 / s, s, rng)
    nu = rng.standard_normal((n, n)) * (0.1 / np.sqrt(n))
    t = np.triu(nu * np.sqrt(np.outer(lam, lam)), 1) + np.diag(lam)
    return np.asfortranarray(q @ t @ q.T)


def selector_params(index: int, n_max_nonsym: int = 1024):
    """Parameters of matrix `index` of the selector's law: (kind, n, kappa,
    seed).  50% SPD and 50% nonsymmetric, n = round(exp(U(ln 64, ln 1024)))
    (nonsymmetric capped at n_max_nonsym), kappa = 10^U(1, 8); nonsymmetric
    inputs are 25% of the 2 I + G / sqrt(n) family and 75% nonsym_kappa."""
    rng = _rng(1_000_003 * (index + 1))
    n = int(round(np.exp(rng.uniform(np.log(64.0), np.log(1024.0)))))
    kappa = float(10.0 ** rng.uniform(1.0, 8.0))
    seed = int(rng.integers(1, 2 ** 31))
    if rng.uniform() < 0.5:
        return "spd", n, kappa, seed
    n = min(n, n_max_nonsym)
    if rng.uniform() < 0.25:
        return "shifted", n, kappa, seed
    return "kappa", n, kappa, seed


def selector_matrix(index: int, n_max_nonsym: int = 1024):
    """One matrix of the selector's training / evaluation law (see
    selector_params).  Returns (A, kind, n, kappa) with kind in {"spd",
    "shifted", "kappa"}."""
    kind, n, kappa, seed = selector_params(index, n_max_nonsym)
    if kind == "spd":
        a, _, _ = spd(n, kappa, seed)
        return a, kind, n, kappa
    if kind == "shifted":
        return nonsym_shifted(n, seed), kind, n, kappa
    return nonsym_kappa(n, kappa, seed), kind, n, kappa