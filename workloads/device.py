"""Device-side versions of the seeded constructions, for the large selector
datasets (thousands of Haar-orthogonal matrices, where host QR dominates).

Same laws as the host generators in this package (Haar Q from the QR of a
Gaussian matrix with the signs of diag(R) folded in; eigenvalues log-uniform
with both endpoints pinned; the same nonsymmetric families), drawn with
torch's generator on the device, seeded per matrix.  The values differ from
the host generators' for the same seed; the parameters of selector matrix
`index` (kind, n, kappa, seed) are the host ones.  Nothing here computes any
part of the square-root method.
"""

from __future__ import annotations

import numpy as np

from . import selector_params


def _gen(seed: int, device):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def haar_orthogonal(n: int, g, device):
    import torch
    z = torch.randn(n, n, generator=g, device=device, dtype=torch.float64)
    q, r = torch.linalg.qr(z)
    d = torch.sign(torch.diagonal(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def loguniform_eigs(n: int, lo: float, hi: float, g, device):
    import torch
    if n == 1:
        return torch.full((1,), float(np.sqrt(lo * hi)), device=device, dtype=torch.float64)
    u = torch.rand(n, generator=g, device=device, dtype=torch.float64)
    lam = torch.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))
    lam[0] = lo
    lam[-1] = hi
    return torch.sort(lam).values


def spd(n: int, kappa: float, seed: int, device="cuda"):
    """A = Q diag(lam) Q^T, lam log-uniform on [kappa^-1/2, kappa^1/2]."""
    g = _gen(seed, device)
    q = haar_orthogonal(n, g, device)
    s = float(np.sqrt(kappa))
    lam = loguniform_eigs(n, 1.0 / s, s, g, device)
    a = (q * lam[None, :]) @ q.T
    return (0.5 * (a + a.T)).contiguous()


def nonsym_shifted(n: int, seed: int, device="cuda"):
    """A = 2 I + G / sqrt(n)."""
    import torch
    g = _gen(seed, device)
    z = torch.randn(n, n, generator=g, device=device, dtype=torch.float64)
    return (2.0 * torch.eye(n, device=device, dtype=torch.float64) + z / np.sqrt(n)).contiguous()


def nonsym_kappa(n: int, kappa: float, seed: int, device="cuda"):
    """A = Q (L + N) Q^T, L = diag(lam), N_ij = nu_ij sqrt(lam_i lam_j)."""
    import torch
    g = _gen(seed, device)
    q = haar_orthogonal(n, g, device)
    s = float(np.sqrt(kappa))
    lam = loguniform_eigs(n, 1.0 / s, s, g, device)
    nu = torch.randn(n, n, generator=g, device=device, dtype=torch.float64) * (0.1 / np.sqrt(n))
    t = torch.triu(nu * torch.sqrt(torch.outer(lam, lam)), 1) + torch.diag(lam)
    return (q @ t @ q.T).contiguous()


def selector_matrix(index: int, n_max_nonsym: int = 1024, device="cuda"):
    """Matrix `index` of the selector's law, generated on the device:
    (A, kind, n, kappa)."""
    kind, n, kappa, seed = selector_params(index, n_max_nonsym)
    if kind == "spd":
        return spd(n, kappa, seed, device), kind, n, kappa
    if kind == "shifted":
        return nonsym_shifted(n, seed, device), kind, n, kappa
    return nonsym_kappa(n, kappa, seed, device), kind, n, kappa
