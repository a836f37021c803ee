"""Near-critical hopping parameter for the synthetic lattice workloads.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper runs "at essentially kappa critical" (Section 2).  For the synthetic
near-identity SU(3) fields the critical point is found numerically: kappa is
chosen so that the smallest |eigenvalue| of gamma5 M (the smallest singular
value of M) equals a target.  f(kappa) = min |lambda(gamma5 M(kappa))| is not
monotone -- it dips at an avoided crossing and rises again -- so the search
scans for the first dip and bisects on its lower side.

Small lattices use the dense spectrum (exact).  Large lattices use the
smallest eigenvalue of M^dag M (= min |lambda(gamma5 M)|^2) from the plain
Lanczos recurrence, whose smallest Ritz value decreases monotonically to
lambda_min (Cauchy interlacing), with the C transcription of M, and a secant
iteration in kappa on the lower side of the critical point.
``python -m oracle.kappa [small|large]`` writes ``tests/golden/kappa.json``;
it calls only oracle code.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from . import dirac


class DenseG5M:
    """gamma5 M(kappa) = gamma5 (1 - kappa D) with the hopping matrix D built once."""

    def __init__(self, links, dims):
        op = dirac.WilsonOperator(links, dims, 1.0)
        # with kappa = 1: M = 1 - D  =>  D = 1 - M
        self.D = np.eye(op.n, dtype=np.complex128) - dirac.dense(op.M, op.n)
        self.g5 = np.tile(np.array([1, 1, 1, 1, 1, 1, -1, -1, -1, -1, -1, -1], float), op.V)
        self.n = op.n

    def min_abs_eig(self, kappa: float) -> float:
        g = self.g5[:, None] * (np.eye(self.n) - kappa * self.D)
        return float(np.min(np.abs(np.linalg.eigvalsh(g))))


def first_dip(f, lo=0.10, hi=0.17, step=0.002):
    """Scan upward for the first local minimum of f, then refine by golden section."""
    ks = np.arange(lo, hi + 1e-12, step)
    vals = []
    for i, k in enumerate(ks):
        vals.append(f(k))
        if i >= 2 and vals[-2] < vals[-3] and vals[-2] <= vals[-1]:
            a, b = ks[i - 2], ks[i]
            break
    else:
        raise RuntimeError("no dip found in the scanned kappa range")
    g = (np.sqrt(5) - 1) / 2
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = f(c), f(d)
    for _ in range(30):
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = f(d)
    kmin = (a + b) / 2
    return kmin, f(kmin), ks[: len(vals)], np.array(vals)


def bisect_lower(f, target, k_lo, k_dip, rel=0.05, maxit=60):
    """kappa in [k_lo, k_dip] with f(kappa) = target (f decreasing there), to within rel."""
    a, b = k_lo, k_dip
    for _ in range(maxit):
        mid = 0.5 * (a + b)
        fm = f(mid)
        if abs(fm - target) <= rel * target * 0.5:
            return mid, fm
        if fm > target:
            a = mid
        else:
            b = mid
    return mid, fm


def search_small(dims, target, seeds=range(10), eps=0.5, log=print):
    from lattice_inputs import su3_links
    for seed in seeds:
        t0 = time.time()
        op = DenseG5M(su3_links(dims, seed, eps), dims)
        kmin, fmin, ks, vals = first_dip(op.min_abs_eig)
        log(f"seed {seed}: dip min {fmin:.4e} at kappa {kmin:.6f} ({time.time() - t0:.0f}s)")
        if fmin <= target:
            below = ks[vals > target]
            k_lo = float(below[below < kmin].max())
            kappa, fk = bisect_lower(op.min_abs_eig, target, k_lo, kmin)
            return dict(dims=list(dims), seed=int(seed), eps=eps, target=target, kappa=float(kappa),
                        min_abs_eig=float(fk), dip_kappa=float(kmin), dip_min=float(fmin))
    raise RuntimeError("no seed reaches the target")


def lanczos_min_eig(apply, n, seed=0, rtol=1e-4, check=200, max_steps=40000):
    """Smallest eigenvalue of a Hermitian positive definite operator (plain Lanczos, no re-orthogonalisation).

    Returns (theta_min, steps).  Stops when the smallest Ritz value changed by
    less than rtol (relative) over the last ``check`` steps.
    """
    import scipy.linalg as sla
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v /= np.linalg.norm(v)
    vp = np.zeros_like(v)
    beta = 0.0
    al, be = [], []
    last = np.inf
    for j in range(max_steps):
        w = apply(v) - beta * vp
        a = float(np.real(np.vdot(v, w)))
        w -= a * v
        b = float(np.linalg.norm(w))
        al.append(a)
        be.append(b)
        if (j + 1) % check == 0:
            th = float(sla.eigvalsh_tridiagonal(np.array(al), np.array(be[:-1]), select="i",
                                                select_range=(0, 0))[0])
            if abs(last - th) <= rtol * abs(th):
                return th, j + 1
            last = th
        vp, v = v, w / b
        beta = b
    return last, max_steps


def search_large(dims, target, seed=0, eps=0.5, k0=0.140, k1=0.145, rel=0.05, log=print):
    """Secant iteration on f(kappa) = sqrt(lambda_min(M^dag M)) - target, lower side of kappa_c."""
    from lattice_inputs import su3_links
    from .cwilson import CWilson
    U = su3_links(dims, seed, eps)
    n = 12 * int(np.prod(dims))

    def f(kappa):
        t0 = time.time()
        op = CWilson(U, dims, kappa)
        th, steps = lanczos_min_eig(op.MdagM, n)
        val = float(np.sqrt(max(th, 0.0)))
        log(f"kappa {kappa:.7f}: min|lambda| {val:.5e} ({steps} Lanczos steps, {time.time() - t0:.0f}s)")
        return val

    pts = [(k0, f(k0)), (k1, f(k1))]
    for _ in range(8):
        (ka, fa), (kb, fb) = pts[-2], pts[-1]
        if abs(fb - target) <= rel * target:
            return dict(dims=list(dims), seed=int(seed), eps=eps, target=target, kappa=float(kb),
                        min_abs_eig=float(fb), method="lanczos-secant")
        kc = kb + (target - fb) * (kb - ka) / (fb - fa)
        kc = min(kc, kb + 2 * (kb - ka)) if kb > ka else kc
        pts.append((kc, f(kc)))
    raise RuntimeError("secant search did not reach the target")


def main(argv=None):
    argv = argv or ["small"]
    out = os.path.join(os.path.dirname(__file__), "..", "tests", "golden", "kappa.json")
    res = {}
    if os.path.exists(out):
        with open(out) as fh:
            res = json.load(fh)
    if "small" in argv:
        res["4x4x4x4"] = search_small((4, 4, 4, 4), 1e-3)
    if "large" in argv:
        res["16x16x16x32"] = search_large((16, 16, 16, 32), 1e-4, log=lambda m: print(m, flush=True))
    if "precision" in argv:
        res["24x24x24x48"] = search_large((24, 24, 24, 48), 1e-3, log=lambda m: print(m, flush=True))
    if "learned" in argv:
        # the learned-guess workload: one kappa for every field, tuned on the first training field
        res["16x16x16x32/seed10"] = search_large((16, 16, 16, 32), 1e-3, seed=10, k0=0.145, k1=0.1474,
                                                 log=lambda m: print(m, flush=True))
    if "batching" in argv:
        # the four lattices of the multi-lattice work list, links seed 0, each at min|lambda| = 1e-3
        for dims in ((8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32), (20, 20, 20, 40)):
            name = "x".join(map(str, dims)) + "/batching"
            res[name] = search_large(dims, 1e-3, k0=0.145, k1=0.1474, log=lambda m: print(m, flush=True))
            with open(out, "w") as fh:
                json.dump(res, fh, indent=1, sort_keys=True)
    if "ksweep" in argv:
        res["20x20x20x32"] = search_large((20, 20, 20, 32), 1e-3, k0=0.145, k1=0.1474,
                                          log=lambda m: print(m, flush=True))
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1, sort_keys=True)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main(sys.argv[1:])
