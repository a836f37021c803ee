"""Benchmark: later right-hand sides per second to rel. residual 1e-10, plus Wilson Dslash HBM GB/s.

Workload (one GPU), the learned-guess held-out set: 16^3 x 32 Wilson lattices with links
U = exp(0.5 i X), one kappa tuned on links seed 10 to min|lambda(gamma5 M)| = 1e-3; training
fields 10-17, held-out fields 20-23.  Setup, untimed and reported separately: Lan-DR(m,k) on
M^dag M for a Gaussian first right-hand side of every field (eigenvectors lowered to FP32),
256 Gaussian (b, x) pairs per training field solved to tol by the batched path, and the
network trained on them in FP32 on the GPU with the loss on the error the D-CG projection
leaves.  One timed step: D-CG for the 4 held-out fields x 64 Gaussian right-hand sides (each
field's 64 in one batch) on the fast path: BF16 Krylov vectors and stencil spinors, FP32
arithmetic and links, FP64 reliable updates, true residuals and solutions, the Galerkin
projection over the field's FP32-rounded eigenvectors and the learned guess, every rhs verified
by its FP64 true residual <= 1e-10.  Inputs and outputs stay in HBM (torch complex128 device
tensors passed as device pointers).  After it: an ablation (storage, eigenvector precision,
network) and the baseline, plain FP64 D-CG one rhs at a time over the same eigenvectors and rhs.

value = 256 * steps / timed seconds (RHS/s).  roofline: the batched BF16 stencil, its average
launch duration taken with HIP events on the library's stream around every launch inside the
timed region; algorithmic bytes per launch = 288 B/site (FP32 links once) + 96 B/site per active
rhs (BF16 input and output spinor).  cpu_baseline: the oracle's D-CG on the host cores for a
bounded sample of the same workload.  c2: the plain-method configuration (16^3 x 32 at
min|lambda| = 1e-4, MinRes-DR then batched D-MinRes on 12 point sources) as extra keys.
Study modes (--multi, --precision, --ksweep, --learned, --window-sweep) print their own line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "RHS/s to rel.res 1e-10 (learned+mixed+batched vs plain FP64); Dslash HBM GB/s"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kappa_for(name):
    with open(os.path.join(ROOT, "tests", "golden", "kappa.json")) as fh:
        return json.load(fh)[name]


def point_sources(dims):
    from lattice_inputs import point_source
    return np.stack([point_source(dims, 0, s, c) for s in range(4) for c in range(3)])


def wilson_source_hash():
    h = hashlib.sha256()
    for f in ("wilson.hip", "cplx.hpp"):
        with open(os.path.join(ROOT, "paper_0901_3163_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(dims, storage, nrhs=12):
    """HBM bytes per Wilson launch from the committed rocprofv3 counter summary, if current."""
    p = os.path.join(ROOT, "profiles", f"wilson_{storage}_nrhs{nrhs}_{'x'.join(map(str, dims))}_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        t = json.load(fh)
    if t.get("source_hash") != wilson_source_hash() or tuple(t.get("dims", ())) != tuple(dims):
        return None
    return t.get("bytes_per_launch")


def pretune_projection(ctx, deflan, n, k, nrhs):
    """Tune (untimed) the contraction shapes the batched projection over k eigenvectors uses for
    nrhs right-hand sides of fields of n complex numbers: the FP64 dots in 64-vector chunks and
    the matrix-core dots in 128-vector chunks, for 16-column groups, and the updates."""
    nws = sorted({min(16, nrhs - c0) for c0 in range(0, nrhs, 16)})
    for nw in nws:
        for j0 in range(0, k, 64):
            ctx.tune_tsk(deflan.DL_TSK_DOTS64, n, min(64, k - j0), nw)
        for j0 in range(0, k, 128):
            ctx.tune_tsk(deflan.DL_TSK_DOTS32, n, min(128, k - j0), nw)
            ctx.tune_tsk(deflan.DL_TSK_DOTS16, n, min(128, k - j0), nw)
        ctx.tune_tsk(deflan.DL_TSK_UPD64, n, k, nw)
        ctx.tune_tsk(deflan.DL_TSK_UPD32, n, k, nw)


def tiled_links(dims, seed=0):
    """SU(3) links for a large lattice: a seeded 8^4 field repeated periodically (values only
    matter for bandwidth, and every link is still an SU(3) matrix)."""
    from lattice_inputs import su3_links
    small = (8, 8, 8, 8)
    u = su3_links(small, seed).reshape(small[3], small[2], small[1], small[0], 4, 3, 3)
    reps = (dims[3] // 8, dims[2] // 8, dims[1] // 8, dims[0] // 8, 1, 1, 1)
    return np.ascontiguousarray(np.tile(u, reps).reshape(-1, 4, 3, 3))


def dslash_sweep(ctx, deflan, sizes, reps):
    """HBM GB/s of the Wilson stencil on lattices above the 256 MB Infinity Cache (event-timed)."""
    import torch
    out = {}
    for dims in sizes:
        V = int(np.prod(dims))
        U = torch.from_numpy(tiled_links(dims)).cuda()
        op = deflan.Operator(ctx, dims, U, 0.13, deflan.DL_G5M)
        del U
        torch.cuda.empty_cache()
        for prec, pname in ((deflan.DL_FP64, "fp64"), (deflan.DL_FP32, "fp32"), (deflan.DL_BF16, "bf16")):
            for nrhs in (1, 12):
                key = f"{'x'.join(map(str, dims))}/{pname}/nrhs{nrhs}"
                out[key] = dslash_point(op, deflan, prec, nrhs, reps)
        op.close()
        torch.cuda.empty_cache()
    return out


def dslash_point(op, deflan, prec, nrhs, reps):
    """One stencil configuration: tuned launch shape, event-timed average over reps launches."""
    variant, order, _ = op.tune_wilson(prec, nrhs, reps=5)  # the project's autotuner
    op.bench_wilson(deflan.DL_APPLY_M, prec, nrhs, 2)  # warm-up
    ms, by = op.bench_wilson(deflan.DL_APPLY_M, prec, nrhs, reps)
    gbs = by / (ms * 1e-3) / 1e9
    log(f"dslash {'x'.join(map(str, op.dims))} prec {prec} nrhs {nrhs}: {ms * 1e3:.1f} us/launch, {gbs:.0f} GB/s")
    return dict(bytes_per_launch=by, avg_us=round(ms * 1e3, 1), GBps=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4),
                working_set_MB=round(by / 1e6, 1), cache_resident=by < 256e6, tuned_variant=variant,
                tuned_order=order)


def copy_ceiling(ctx, nbytes=1 << 30, reps=20):
    """The library's streaming copy kernel over 1 GiB (read + write): the practical HBM ceiling."""
    ctx.bench_copy(nbytes, 2)
    ms = ctx.bench_copy(nbytes, reps)
    gbs = 2.0 * nbytes / (ms * 1e-3) / 1e9
    log(f"copy kernel: {gbs:.0f} GB/s over {nbytes >> 20} MiB")
    return dict(bytes_per_launch=2 * nbytes, avg_us=round(ms * 1e3, 1), GBps=round(gbs, 1),
                frac=round(gbs / HBM_PEAK_GBS, 4))


def cpu_baseline(dims, kappa, iters_per_rhs, k):
    """Oracle D-MinRes on the host cores: one point source, projection + 200 MinRes iterations."""
    from lattice_inputs import point_source, su3_links
    from oracle import cwilson, deflated, krylov
    cores = len(os.sched_getaffinity(0))
    U = su3_links(dims, 0)
    op = cwilson.CWilson(U, dims, kappa)
    n = op.n
    rng = np.random.default_rng(7)
    Y, _ = np.linalg.qr(rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k)))
    b = point_source(dims, 0, 0, 0).ravel()
    t0 = time.time()
    H = deflated.projection_matrix(op.g5M, Y)  # once per handle, not per rhs
    t_h = time.time() - t0
    nit = 200
    t0 = time.time()
    bA = np.where(np.tile([1] * 6 + [-1] * 6, n // 12) > 0, b, -b)  # gamma5 b
    x0 = deflated.galerkin_projection(Y, H, bA)
    t_proj = time.time() - t0
    t0 = time.time()
    krylov.minres(op.g5M, bA, x0=x0, tol=0.0, maxiter=nit)
    t_it = (time.time() - t0) / nit
    per_rhs = t_proj + iters_per_rhs * t_it
    return dict(value=round(1.0 / per_rhs, 5), unit="RHS/s", cores=cores, kind="oracle",
                sample=(f"oracle D-MinRes (numpy vectors, OpenMP C Wilson matrix) on {'x'.join(map(str, dims))}: "
                        f"Galerkin projection over {k} seeded orthonormal vectors ({t_proj:.2f}s) + {nit} MinRes "
                        f"iterations ({t_it * 1e3:.1f} ms/iter) on one point source; per-rhs time = projection + "
                        f"{iters_per_rhs:.0f} iterations (the GPU run's mean per rhs); H = Y^H A Y setup "
                        f"({t_h:.1f}s) excluded like the GPU's"),
                seconds_per_rhs=round(per_rhs, 3))


def train_guess(ctx, op, eig, deflan, dims, args):
    """Train the learned-guess network on (b, x) pairs of the benchmark field: b = point
    sources at seeded random sites other than site 0 (random spin and colour), x from the
    batched mixed-precision D-MinRes to the benchmark tolerance.  Returns (net, summary)."""
    import torch
    from lattice_inputs import net_weights, point_source
    V = int(np.prod(dims))
    rng = np.random.default_rng(900)
    sites = rng.choice(np.arange(1, V), size=args.train_rhs, replace=False)
    Bt = np.stack([point_source(dims, int(s), int(rng.integers(4)), int(rng.integers(3))) for s in sites])
    Bt = torch.from_numpy(Bt).cuda()
    t0 = time.time()
    Xt, st, _ = op.solve_next(Bt, eig, args.tol, storage=deflan.DL_FP32, batched=1)
    torch.cuda.synchronize()
    t_pairs = time.time() - t0
    log(f"learned guess: {args.train_rhs} training pairs solved in {t_pairs:.1f}s")
    net = deflan.Net(ctx, net_weights(args.net_seed))
    t0 = time.time()
    losses = net.train(op, Bt, Xt, batch=args.train_batch, steps=args.train_steps, lr=args.train_lr)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    log(f"learned guess: {args.train_steps} Adam steps in {t_train:.1f}s, loss {losses[0]:.4f} -> "
        f"{np.mean(losses[-10:]):.4f}")
    del Bt, Xt
    info = dict(training_pairs=args.train_rhs, pair_seconds=round(t_pairs, 2), steps=args.train_steps,
                batch=args.train_batch, lr=args.train_lr, train_seconds=round(t_train, 2),
                loss_first=round(float(losses[0]), 5), loss_last10=round(float(np.mean(losses[-10:])), 5),
                pairs="point sources at seeded random sites != 0 of the benchmark field, x from batched "
                      "FP32/FP64 D-MinRes at the benchmark tolerance",
                loss="mean ||M (net(b) - x)||^2 / ||b||^2")
    return net, info


def projection_sweep(ctx, deflan, shapes, reps):
    """The deflation contraction C = V^H W (k eigenvectors against 12 columns) on device fields:
    FP64 (LDS tiles, vector FMAs) and FP32 / BF16 storage on the matrix cores.  Kernel time from
    HIP events around the contraction launches only; algorithmic bytes = every basis vector and
    every column read once; useful flops = 8 k * 12 * n (complex multiply-add)."""
    import torch
    out = {}
    nw = 12
    for dims, k in shapes:
        n = 12 * int(np.prod(dims))
        g = torch.Generator(device="cuda")
        g.manual_seed(1)
        V = torch.randn(k, n, dtype=torch.complex128, device="cuda", generator=g)
        W = torch.randn(nw, n, dtype=torch.complex128, device="cuda", generator=g)
        for name, prec, bpc in (("fp64", None, 16), ("fp32", deflan.DL_FP32, 8), ("bf16", deflan.DL_BF16, 4)):
            def call():
                if prec is None:
                    return deflan.dl_tsk_project_multi(ctx, V, W)
                return deflan.dl_tsk_project_lowp(ctx, prec, V, W)
            call()
            torch.cuda.synchronize()
            ctx.timing(True)
            for _ in range(reps):
                call()
            nl, ms, _ = ctx.kernel_time("tsk_dots")
            ctx.timing(False)
            t = ms / reps * 1e-3
            by = (k + nw) * n * bpc
            gbs = by / t / 1e9
            key = f"{'x'.join(map(str, dims))}/k{k}/{name}"
            out[key] = dict(k=k, nrhs=nw, launches_per_call=nl / reps, us_per_call=round(t * 1e6, 1),
                            GBps=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4),
                            useful_TFLOPs=round(8.0 * k * nw * n / t / 1e12, 2),
                            engine="matrix cores (MFMA)" if prec is not None else "vector FMA")
            log(f"projection {key}: {t * 1e6:.1f} us, {gbs:.0f} GB/s")
        del V, W
        torch.cuda.empty_cache()
    return out


def precision_study(args):
    """The precision ablation on the 24^3x48 near-critical lattice (min|lambda(gamma5 M)| ~ 1e-3):
    FP64 Lan-DR(200,100) on M^dag M for a Gaussian first rhs (seed 299), the eigenvectors
    lowered to FP32 and BF16, then D-CG for 12 Gaussian rhs (seeds 300-311) on the batched path
    with FP32 or BF16 Krylov storage (FP32 arithmetic, FP64 restarts; reliable updates every 50
    iterations with FP32, the BF16 D-CG defaults with BF16) and the projection over FP64 or FP32
    eigenvectors.  Each
    case: RHS/s, iterations, the library's FP64 true residual and the relative error against
    the plain FP64 D-CG solutions of the same rhs on the GPU (the parity-checked FP64 path).
    Prints one JSON line."""
    import torch
    from lattice_inputs import gaussian_spinor, su3_links
    from paper_0901_3163_amd import deflan
    os.environ.setdefault("DEFLAN_VERBOSE", "1")
    try:
        e = kappa_for("24x24x24x48")
    except KeyError:
        sys.exit("no kappa stored for 24x24x24x48: run `python -m oracle.kappa precision`")
    dims, kappa, tol = tuple(e["dims"]), e["kappa"], args.tol
    ctx = deflan.Context(0)
    U = torch.from_numpy(su3_links(dims, e["seed"], e["eps"])).cuda()
    op = deflan.Operator(ctx, dims, U, kappa, deflan.DL_MDAGM)
    del U
    log(f"precision study 24^3x48 kappa {kappa:.7f}: Lan-DR({args.prec_m},{args.prec_k})")
    t0 = time.time()
    _, eig, st1 = op.solve_first(torch.from_numpy(gaussian_spinor(dims, 299)).cuda(), args.prec_m, args.prec_k, tol,
                                 reorth=deflan.DL_REORTH_KEPT if args.reorth == "kept" else deflan.DL_REORTH_FULL)
    torch.cuda.synchronize()
    t_first = time.time() - t0
    log(f"first rhs: {st1['mvp']} MVPs, {t_first:.1f}s, relres {st1['relres']:.2e}")
    t0 = time.time()
    lower_mvp = eig.lower(deflan.DL_FP32)
    torch.cuda.synchronize()
    t_lower = time.time() - t0
    B = torch.from_numpy(np.stack([gaussian_spinor(dims, 300 + i) for i in range(12)])).cuda()
    nrhs = B.shape[0]
    pretune_projection(ctx, deflan, 12 * int(np.prod(dims)), args.prec_k, nrhs)
    t0 = time.time()
    X64, st64, _ = op.solve_next(B, eig, tol)
    torch.cuda.synchronize()
    t64 = time.time() - t0
    log(f"plain FP64 D-CG: {nrhs / t64:.2f} RHS/s, iters {np.mean([s['iters'] for s in st64]):.0f}")
    nx = torch.linalg.vector_norm(X64.reshape(nrhs, -1), dim=1)
    cases = {}
    for sname, scode in (("fp32", deflan.DL_FP32), ("bf16", deflan.DL_BF16)):
        # reliable updates every 50 iterations with FP32 storage; BF16 takes the library's BF16
        # D-CG settings (updates every 8 iterations in 1e-5 cycles from the projection-only start)
        rel = 50 if scode == deflan.DL_FP32 else None
        op.solve_next(B, eig, tol, storage=scode, batched=1, reliable_every=rel)  # tuning and warm-up, 12 rhs
        # (the BF16 contraction serves the gamma5 M form only: on M^dag M its error reaches the
        # residual amplified by 1/sigma_min(M))
        for ename, ecode in (("fp64", deflan.DL_FP64), ("fp32", deflan.DL_FP32)):
            torch.cuda.synchronize()
            t0 = time.time()
            X, sts, rc = op.solve_next(B, eig, tol, storage=scode, batched=1, reliable_every=rel, eig_storage=ecode)
            torch.cuda.synchronize()
            dt = time.time() - t0
            err = torch.linalg.vector_norm((X - X64).reshape(nrhs, -1), dim=1) / nx
            key = f"storage_{sname}/eig_{ename}"
            cases[key] = dict(value=round(nrhs / dt, 3), unit="RHS/s", seconds=round(dt, 3),
                              iters_per_rhs=float(np.mean([s["iters"] for s in sts])),
                              max_relres=float(max(s["relres"] for s in sts)),
                              all_rhs_converged=bool(rc == 0 and all(s["relres"] <= tol for s in sts)),
                              max_rel_error_vs_fp64_path=float(err.max()))
            log(f"{key}: {nrhs / dt:.2f} RHS/s, iters {cases[key]['iters_per_rhs']:.0f}, "
                f"err {cases[key]['max_rel_error_vs_fp64_path']:.1e}")
    n = 12 * int(np.prod(dims))
    res = dict(workload=(f"24^3x48 Wilson near-critical (kappa {kappa:.6f}), Lan-DR({args.prec_m},{args.prec_k}) "
                         f"on M^dag M, then D-CG on 12 Gaussian rhs, tol {tol:g}"),
               first_rhs=dict(mvp=st1["mvp"], mvp_lin=st1["mvp_lin"], seconds=round(t_first, 2),
                              relres=st1["relres"], stop_rule=st1["stop_rule"]),
               lowering=dict(mvp=lower_mvp, seconds=round(t_lower, 2)),
               eigenvector_bytes=dict(fp64=args.prec_k * n * 16, fp32=args.prec_k * n * 8),
               plain_fp64=dict(value=round(nrhs / t64, 3), unit="RHS/s",
                               iters_per_rhs=float(np.mean([s["iters"] for s in st64])),
                               max_relres=float(max(s["relres"] for s in st64))),
               cases=cases,
               error_reference="plain FP64 D-CG on the GPU (one rhs at a time), the path the parity tests check "
                               "against the oracle")
    eig.close()
    op.close()
    ctx.close()
    print(json.dumps(res), flush=True)


def learned_study(args):
    """The learned initial guess across gauge fields: 16^3x32, training fields with links seeds
    10-17, held-out fields 20-23, all at the benchmark kappa (tuned on seed 0).  Per field the
    first rhs (Gaussian) runs MinRes-DR(m,k) on gamma5 M; the training pairs are 256 Gaussian rhs
    per training field (2048 in all) solved to tol by the batched path; the network is trained
    in FP32 by Adam, cycling over the training fields; each held-out field then solves 64 Gaussian
    rhs (in batches of 16) from net(b) + projection and from the projection alone.  The path is
    the benchmark's (batched D-MinRes, BF16 storage, BF16-contracted projection).  Prints one JSON
    line."""
    import torch
    from lattice_inputs import gaussian_spinor, net_weights, su3_links
    from paper_0901_3163_amd import deflan
    e = kappa_for("16x16x16x32")
    dims, kappa, tol = tuple(e["dims"]), e["kappa"], args.tol
    ctx = deflan.Context(0)
    st_, est = deflan.DL_BF16, deflan.DL_BF16
    per_train, per_test, bs = args.learned_pairs, args.learned_test, 16

    def field(seed):
        U = torch.from_numpy(su3_links(dims, seed, e["eps"])).cuda()
        op = deflan.Operator(ctx, dims, U, kappa, deflan.DL_G5M)
        del U
        t0 = time.time()
        _, eig, st1 = op.solve_first(torch.from_numpy(gaussian_spinor(dims, 1000 + seed)).cuda(), args.m, args.k, tol)
        eig.lower(est)
        torch.cuda.synchronize()
        log(f"learned: field {seed}: MinRes-DR({args.m},{args.k}) {st1['mvp']} MVPs, {time.time() - t0:.1f}s")
        return op, eig, dict(seed=seed, first_rhs_mvp=st1["mvp"], first_rhs_seconds=round(time.time() - t0, 2))

    def rhs(seed0, n):
        return torch.from_numpy(np.stack([gaussian_spinor(dims, seed0 + i) for i in range(n)])).cuda()

    def solve(op, eig, B, net=None, nprec=deflan.DL_FP32):
        its, kept, ok = [], [], True
        t0 = time.time()
        X = torch.empty_like(B)
        for i in range(0, B.shape[0], bs):
            Xi, sts, rc = op.solve_next(B[i:i + bs], eig, tol, storage=st_, batched=1, net=net, eig_storage=est,
                                        net_prec=nprec)
            X[i:i + bs] = Xi
            its += [s["iters"] for s in sts]
            kept += [s["guess"] for s in sts]
            ok &= rc == 0 and all(s["relres"] <= tol for s in sts)
        torch.cuda.synchronize()
        return X, its, kept, ok, time.time() - t0

    train, fields_info = [], []
    t_pairs = 0.0
    for seed in range(10, 18):
        op, eig, info = field(seed)
        B = rhs(20000 + 1000 * seed, per_train)
        X, its, _, ok, dt = solve(op, eig, B)
        t_pairs += dt
        info.update(pairs=per_train, pair_iters_per_rhs=float(np.mean(its)), pairs_converged=bool(ok))
        fields_info.append(info)
        eig.close()
        train.append((op, B, X))
        log(f"learned: field {seed}: {per_train} pairs in {dt:.1f}s, {np.mean(its):.0f} iterations per rhs")
    net = deflan.Net(ctx, net_weights(args.net_seed))
    t0 = time.time()
    losses = []
    for ep in range(args.learned_epochs):
        for op, B, X in train:
            losses += list(net.train(op, B, X, batch=args.train_batch, steps=args.learned_steps, lr=args.train_lr))
    torch.cuda.synchronize()
    t_train = time.time() - t0
    log(f"learned: {len(losses)} Adam steps in {t_train:.1f}s, loss {losses[0]:.4f} -> {np.mean(losses[-20:]):.4f}")
    for op, B, X in train:
        op.close()
    del train
    torch.cuda.empty_cache()
    held = []
    for seed in range(20, 24):
        op, eig, info = field(seed)
        B = rhs(40000 + 1000 * seed, per_test)
        solve(op, eig, B[:bs])  # launch-shape tuning and warm-up
        X0, it0, _, ok0, dt0 = solve(op, eig, B)
        X1, it1, kept, ok1, dt1 = solve(op, eig, B, net)
        _, it2, kept2, ok2, dt2 = solve(op, eig, B, net, deflan.DL_BF16)
        nx = torch.linalg.vector_norm(X0.reshape(per_test, -1), dim=1)
        diff = float((torch.linalg.vector_norm((X1 - X0).reshape(per_test, -1), dim=1) / nx).max())
        held.append(dict(info, rhs=per_test, projection_only=dict(value=round(per_test / dt0, 3), unit="RHS/s",
                                                                   iters_per_rhs=float(np.mean(it0)),
                                                                   all_rhs_converged=bool(ok0)),
                         net_plus_projection=dict(value=round(per_test / dt1, 3), unit="RHS/s",
                                                  iters_per_rhs=float(np.mean(it1)), all_rhs_converged=bool(ok1),
                                                  guess_kept=float(np.mean(kept)), inference="fp32"),
                         net_bf16_plus_projection=dict(value=round(per_test / dt2, 3), unit="RHS/s",
                                                       iters_per_rhs=float(np.mean(it2)),
                                                       all_rhs_converged=bool(ok2),
                                                       guess_kept=float(np.mean(kept2)), inference="bf16"),
                         max_rel_difference_of_solutions=diff))
        log(f"learned: held-out field {seed}: iterations {np.mean(it0):.1f} -> {np.mean(it1):.1f} "
            f"(BF16 inference {np.mean(it2):.1f}), RHS/s {per_test / dt0:.1f} -> {per_test / dt1:.1f} "
            f"(BF16 inference {per_test / dt2:.1f})")
        eig.close()
        op.close()
    res = dict(workload=(f"16^3x32 Wilson (kappa {kappa:.6f} for every field), training fields 10-17, held-out 20-23, "
                         f"Gaussian rhs, batched D-MinRes BF16 with BF16-contracted projection, tol {tol:g}"),
               training=dict(fields=fields_info, pairs=per_train * 8, pair_seconds=round(t_pairs, 2),
                             epochs=args.learned_epochs, steps_per_field=args.learned_steps,
                             batch=args.train_batch, lr=args.train_lr, adam_steps=len(losses),
                             train_seconds=round(t_train, 2), loss_first=round(float(losses[0]), 5),
                             loss_last20=round(float(np.mean(losses[-20:])), 5)),
               held_out=held,
               iters_saved_per_rhs=float(np.mean([h["projection_only"]["iters_per_rhs"]
                                                  - h["net_plus_projection"]["iters_per_rhs"] for h in held])))
    net.close()
    ctx.close()
    print(json.dumps(res), flush=True)


def ksweep_study(args):
    """The paper's k-sweep on a 20^3x32 near-critical field (Section 3, Figs. 5 and 6): for the
    first rhs, unrestarted CG on the normal equations and MinRes on gamma5 M against
    Lan-DR(200, k) and MinRes-DR(200, k) for k = 20, 60, 150 (MVPs to a relative residual of 1e-8
    when the linear system converges, and in all, the run continuing for the eigenvectors); for a
    second rhs, D-CG and D-MinRes with each k against plain CG and MinRes.  All FP64, one rhs at a
    time, MVPs as in the paper (M^dag M counts 2).  Prints one JSON line."""
    import torch
    from lattice_inputs import gaussian_spinor, su3_links
    from paper_0901_3163_amd import deflan
    os.environ.setdefault("DEFLAN_VERBOSE", "1")
    try:
        e = kappa_for("20x20x20x32")
    except KeyError:
        sys.exit("no kappa stored for 20x20x20x32: run `python -m oracle.kappa ksweep`")
    dims, kappa, tol, m = tuple(e["dims"]), e["kappa"], 1e-8, 200
    ctx = deflan.Context(0)
    U = torch.from_numpy(su3_links(dims, e["seed"], e["eps"])).cuda()
    b1 = torch.from_numpy(gaussian_spinor(dims, 500)).cuda()
    b2 = torch.from_numpy(gaussian_spinor(dims, 501)).cuda()[None]
    out = dict(workload=(f"20^3x32 Wilson near-critical (kappa {kappa:.6f}, min|lambda(gamma5 M)| "
                         f"{e['min_abs_eig']:.2e}), m = {m}, tol {tol:g}, FP64"), methods={})
    for name, kind, first, nxt in (("M^dag M", deflan.DL_MDAGM, "Lan-DR", "D-CG"),
                                   ("gamma5 M", deflan.DL_G5M, "MinRes-DR", "D-MinRes")):
        op = deflan.Operator(ctx, dims, U, kappa, kind)
        _, s_p1, _ = op.solve_next(b1[None], None, tol)  # unrestarted CG / MinRes
        _, s_plain, _ = op.solve_next(b2, None, tol)
        plain = "CG" if kind == deflan.DL_MDAGM else "MinRes"
        res = dict(plain_first_rhs=dict(method=plain, mvp=s_p1[0]["mvp"], iters=s_p1[0]["iters"]),
                   plain_second_rhs=dict(method=plain, mvp=s_plain[0]["mvp"], iters=s_plain[0]["iters"]), k={})
        log(f"ksweep {name}: {plain} {s_p1[0]['mvp']} MVPs on the first rhs, {s_plain[0]['mvp']} on a second")
        for k in (20, 60, 150):
            t0 = time.time()
            _, eig, st1 = op.solve_first(b1, m, k, tol)
            torch.cuda.synchronize()
            t1 = time.time() - t0
            _, s2, _ = op.solve_next(b2, eig, tol)
            ev, rs = eig.info()
            res["k"][str(k)] = dict(first_rhs=dict(method=f"{first}({m},{k})", mvp_to_tol=st1["mvp_lin"],
                                                   mvp=st1["mvp"], stop_rule=st1["stop_rule"],
                                                   seconds=round(t1, 2)),
                                    second_rhs=dict(method=nxt, mvp=s2[0]["mvp"], iters=s2[0]["iters"]),
                                    smallest_abs_eigenvalue=float(np.min(np.abs(ev))),
                                    largest_kept_abs_eigenvalue=float(np.max(np.abs(ev))),
                                    max_eigen_residual=float(np.max(rs)))
            log(f"ksweep {name} k={k}: {first} {st1['mvp_lin']} MVPs to tol ({st1['mvp']} in all, {t1:.1f}s); "
                f"{nxt} {s2[0]['mvp']} MVPs")
            if kind == deflan.DL_G5M and k == 150:
                # CG on the indefinite gamma5 M with and without these eigenvectors (Section 3, Fig. 7)
                _, sc0, rc0 = op.solve_next(b1[None], None, tol, method=deflan.DL_METHOD_CG)
                _, sc1, rc1 = op.solve_next(b2, eig, tol, method=deflan.DL_METHOD_CG)
                res["cg_on_gamma5_m"] = dict(first_rhs=dict(mvp=sc0[0]["mvp"], converged=bool(rc0 == 0)),
                                             second_rhs_deflated_k150=dict(mvp=sc1[0]["mvp"],
                                                                           converged=bool(rc1 == 0)))
                log(f"ksweep gamma5 M: CG {sc0[0]['mvp']} MVPs, D-CG (k=150) {sc1[0]['mvp']} MVPs")
            eig.close()
        out["methods"][name] = res
        op.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def multi_lattice(args):
    """Uneven lattices in one batched solve: 16 Gaussian rhs on each of 8^4, 12^4, 16^3x32 and
    20^3x40 (64 in all), D-CG on M^dag M with k = 40, 60, 80, 100 eigenvectors from Lan-DR(k + 40, k)
    (setup, untimed).  Timed, each after a warm-up: one dl_solve_next_multi over all 64 rhs with
    either stencil form (one work-list launch, or one tuned launch per lattice), with and
    without graph replay; the same rhs as four per-lattice batched calls; plain FP64 D-CG on 2
    rhs per lattice (per-rhs time, scaled to 16 rhs).  Prints one JSON line."""
    import torch
    from lattice_inputs import gaussian_spinor, su3_links
    from paper_0901_3163_amd import deflan
    os.environ.setdefault("DEFLAN_VERBOSE", "1")
    storage = {"fp32": deflan.DL_FP32, "bf16": deflan.DL_BF16}[args.multi_storage]
    kappa, tol = 0.145, args.tol
    lats = [((8, 8, 8, 8), 40), ((12, 12, 12, 12), 60), ((16, 16, 16, 32), 80), ((20, 20, 20, 40), 100)]
    # --multi-critical: links seed 0 of each lattice at its own kappa for min|lambda(gamma5 M)| = 1e-3
    crit = {"x".join(map(str, d)): kappa_for("x".join(map(str, d)) + "/batching") for d, _ in lats} \
        if args.multi_critical else None
    ctx = deflan.Context(0)
    items, setup = [], {}
    seed = 400
    for j, (dims, k) in enumerate(lats):
        name = "x".join(map(str, dims))
        kap = crit[name]["kappa"] if crit else kappa
        U = torch.from_numpy(su3_links(dims, 0 if crit else 10 + j)).cuda()
        op = deflan.Operator(ctx, dims, U, kap, deflan.DL_MDAGM)
        del U
        t0 = time.time()
        b1 = torch.from_numpy(gaussian_spinor(dims, 300 + j)).cuda()
        _, eig, st1 = op.solve_first(b1, k + 40, k, tol,
                                     reorth=deflan.DL_REORTH_KEPT if args.reorth == "kept" else deflan.DL_REORTH_FULL)
        torch.cuda.synchronize()
        setup[name] = dict(k=k, kappa=kap, first_rhs_mvp=st1["mvp"], first_rhs_seconds=round(time.time() - t0, 2))
        if crit:
            setup[name]["min_abs_eig"] = crit[name]["min_abs_eig"]
        log(f"multi: {name} Lan-DR({k + 40},{k}) done, {st1['mvp']} MVPs")
        B = torch.from_numpy(np.stack([gaussian_spinor(dims, seed + i) for i in range(16)])).cuda()
        seed += 16
        items.append((op, eig, B, tol))
    nrhs = 16 * len(lats)
    out = {}
    # one batched solve over all lattices; its stencil stage either one work-list launch over
    # every lattice ("list") or one launch per lattice in that lattice's tuned shape ("lattice"),
    # the library's choice by timing unless DEFLAN_MULTI_STENCIL forces one; every other stage
    # is one launch over all 64 rhs
    forced = os.environ.get("DEFLAN_MULTI_STENCIL")
    for form, key in (("list", "one_launch_per_stage"), ("lattice", "per_lattice_stencil_in_one_batch")):
        os.environ["DEFLAN_MULTI_STENCIL"] = form
        for graph in (False, True):
            deflan.solve_next_multi(ctx, items, storage=storage, graph=graph)  # warm-up (tuning, graphs)
            torch.cuda.synchronize()
            t0 = time.time()
            Xs, sts, rc = deflan.solve_next_multi(ctx, items, storage=storage, graph=graph)
            torch.cuda.synchronize()
            dt = time.time() - t0
            ok = rc == 0 and all(s["relres"] <= tol for ss in sts for s in ss)
            out[key + ("_graph" if graph else "")] = dict(
                value=round(nrhs / dt, 3), unit="RHS/s", seconds=round(dt, 3), all_rhs_converged=bool(ok),
                iters_per_rhs=float(np.mean([s["iters"] for ss in sts for s in ss])))
            log(f"multi: one batch over all lattices, stencil form {form} (graph {graph}): {nrhs / dt:.2f} RHS/s")
    if forced is None:
        del os.environ["DEFLAN_MULTI_STENCIL"]
    else:
        os.environ["DEFLAN_MULTI_STENCIL"] = forced
    for op, eig, B, _ in items:  # warm-up of the per-lattice shapes (tuning) as for the work list
        op.solve_next(B, eig, tol, storage=storage, batched=1)
    torch.cuda.synchronize()
    t0 = time.time()
    ok = True
    for op, eig, B, _ in items:
        X, st, rc = op.solve_next(B, eig, tol, storage=storage, batched=1)
        ok &= rc == 0
    torch.cuda.synchronize()
    dt = time.time() - t0
    out["per_lattice_batches"] = dict(value=round(nrhs / dt, 3), unit="RHS/s", seconds=round(dt, 3),
                                      all_rhs_converged=bool(ok))
    log(f"multi: four per-lattice batches: {nrhs / dt:.2f} RHS/s")
    t_plain = 0.0
    for op, eig, B, _ in items:
        op.solve_next(B[:1], eig, tol)  # warm-up (tuning of the one-rhs shapes)
        torch.cuda.synchronize()
        t0 = time.time()
        X, st, rc = op.solve_next(B[:2], eig, tol)
        torch.cuda.synchronize()
        t_plain += (time.time() - t0) * 8  # 2 of 16 rhs
    out["plain_fp64_per_rhs"] = dict(value=round(nrhs / t_plain, 3), unit="RHS/s",
                                     sample="2 rhs per lattice, time scaled to 16")
    kdesc = ("links seed 0, each lattice at its kappa for min|lambda(gamma5 M)| = 1e-3" if crit
             else f"kappa {kappa}")
    res = dict(workload="uneven lattices 8^4, 12^4, 16^3x32, 20^3x40, 16 Gaussian rhs each, D-CG on M^dag M, "
                        f"{kdesc}, tol {tol:g}, {args.multi_storage} storage", setup=setup, **out)
    for op, eig, B, _ in items:
        eig.close()
        op.close()
    ctx.close()
    print(json.dumps(res), flush=True)


def kernel_only(args):
    """The dominant kernel alone, for rocprofv3 counter runs: the stencil of the headline path
    (M, BF16 spinors -- or --storage fp32 -- FP32 links) on held-out field 20 of the learned-guess
    workload (16^3x32) for its 64 right-hand sides at once (reps launches, tuned shape), then the
    library's copy kernel over 1 GiB (reps launches), whose FETCH_SIZE / WRITE_SIZE calibrate the
    counters."""
    import torch
    from lattice_inputs import su3_links
    from paper_0901_3163_amd import deflan
    e = kappa_for("16x16x16x32/seed10")
    dims = tuple(e["dims"])
    nrhs = args.test_rhs
    ctx = deflan.Context(0)
    if args.ko_lattice:
        # an HBM-resident lattice of the sweep instead (links: a seeded 8^4 field tiled)
        dims = tuple(int(v) for v in args.ko_lattice.split("x"))
        links = tiled_links(dims)
    else:
        links = su3_links(dims, 20, e["eps"])
    op = deflan.Operator(ctx, dims, torch.from_numpy(links).cuda(), e["kappa"], deflan.DL_MDAGM)
    del links
    prec = {"fp32": deflan.DL_FP32, "bf16": deflan.DL_BF16}[args.storage]
    op.tune_wilson(prec, nrhs, reps=3)
    ms, by = op.bench_wilson(deflan.DL_APPLY_M, prec, nrhs, args.reps)
    log(f"wilson {args.storage} nrhs{nrhs}: {ms * 1e3:.1f} us/launch, algorithmic {by / 1e6:.1f} MB/launch")
    cms = ctx.bench_copy(1 << 30, args.reps)
    log(f"copy: 1 GiB read + 1 GiB written per launch, {cms * 1e3:.1f} us")
    print(json.dumps(dict(kernel=f"Wilson stencil M, {args.storage} spinors", dims=list(dims), nrhs=nrhs,
                          reps=args.reps, avg_us=round(ms * 1e3, 2), algorithmic_bytes=by,
                          copy_bytes=1 << 30, copy_avg_us=round(cms * 1e3, 2), source_hash=wilson_source_hash())))
    op.close()
    ctx.close()


def tune_report(args):
    """The autotuner's choices at the sizes the paths use: the stencil on the 16^3x32 learned-guess
    field (BF16, FP32 and FP64 spinors with 64 rhs, FP64 with one) and the tall-skinny contractions
    (projection dots and update over k = 60 eigenvectors for 16 rhs, the basis rebuild of
    Lan-DR(120,60) and MinRes-DR(120,60); at 24^3x48 the FP32 projection over k = 100 for 12 rhs
    and the Lan-DR(200,100) rebuild), every key re-timed (run with DEFLAN_VERBOSE=1 for every
    candidate's time).  One JSON line."""
    import torch
    from lattice_inputs import su3_links
    from paper_0901_3163_amd import deflan
    e = kappa_for("16x16x16x32/seed10")
    dims = tuple(e["dims"])
    ctx = deflan.Context(0)
    out = {"stencil": [], "contraction": []}
    op = deflan.Operator(ctx, dims, torch.from_numpy(su3_links(dims, 10, e["eps"])).cuda(), e["kappa"],
                         deflan.DL_MDAGM)
    for prec, nrhs in [(deflan.DL_BF16, 64), (deflan.DL_FP32, 64), (deflan.DL_FP64, 64), (deflan.DL_FP64, 1)]:
        v, o, us = op.tune_wilson(prec, nrhs, reps=10)
        out["stencil"].append(dict(dims=list(dims), prec=prec, nrhs=nrhs, variant=v, order=o, us=round(us, 1)))
        log(f"tune stencil prec {prec} nrhs {nrhs}: variant {v} order {o}, {us:.1f} us")
    op.close()
    n16, n24 = int(np.prod(dims)) * 12, 24 * 24 * 24 * 48 * 12
    for kind, n, nv, nw in [(deflan.DL_TSK_DOTS16, n16, 60, 16), (deflan.DL_TSK_DOTS32, n16, 60, 16),
                            (deflan.DL_TSK_UPD32, n16, 60, 16), (deflan.DL_TSK_DOTS64, n16, 60, 16),
                            (deflan.DL_TSK_UPD64, n16, 60, 16), (deflan.DL_TSK_COMBINE, n16, 120, 60),
                            (deflan.DL_TSK_COMBINE, n16, 121, 61), (deflan.DL_TSK_DOTS32, n24, 100, 12),
                            (deflan.DL_TSK_UPD32, n24, 100, 12), (deflan.DL_TSK_COMBINE, n24, 200, 100)]:
        g, t, us = ctx.tune_tsk(kind, n, nv, nw, reps=5)
        out["contraction"].append(dict(kind=kind, n=n, nv=nv, nw=nw, grid=g, tile=t, us=round(us, 1)))
        log(f"tune contraction {kind} n {n} nv {nv} nw {nw}: grid {g} tile {t}, {us:.1f} us")
    ctx.close()
    print(json.dumps(out))


def projection_only(args):
    """The deflation contraction alone, for rocprofv3 counter runs: C = V^H W for k = 60
    eigenvectors and 12 columns of the 16^3x32 field length, reps calls each in FP64, FP32 and
    BF16 storage (the FP32 / BF16 calls round V and W on the device first)."""
    import torch
    from paper_0901_3163_amd import deflan
    ctx = deflan.Context(0)
    dims, k, nw = (16, 16, 16, 32), 60, 12
    n = 12 * int(np.prod(dims))
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    V = torch.randn(k, n, dtype=torch.complex128, device="cuda", generator=g)
    W = torch.randn(nw, n, dtype=torch.complex128, device="cuda", generator=g)
    res = {}
    for name, prec, bpc in (("fp64", None, 16), ("fp32", deflan.DL_FP32, 8), ("bf16", deflan.DL_BF16, 4)):
        ctx.timing(True)
        for _ in range(args.reps):
            if prec is None:
                deflan.dl_tsk_project_multi(ctx, V, W)
            else:
                deflan.dl_tsk_project_lowp(ctx, prec, V, W)
        nl, ms, _ = ctx.kernel_time("tsk_dots")
        ctx.timing(False)
        res[name] = dict(launches=nl, avg_us_per_call=round(ms / args.reps * 1e3, 1),
                         algorithmic_bytes_per_call=(k + nw) * n * bpc)
        log(f"projection {name}: {ms / args.reps * 1e3:.1f} us per call ({nl // args.reps} launches)")
    print(json.dumps(dict(kernel="deflation contraction C = V^H W", dims=list(dims), k=k, nrhs=nw, reps=args.reps,
                          **res)))
    ctx.close()


def net_only(args):
    """The learned guess's forward pass alone, for rocprofv3 runs: 12 point sources on the 16^3x32
    benchmark field, reps calls each with FP32 inference and with the BF16 matrix-core middle layer."""
    import torch
    from lattice_inputs import net_weights
    from paper_0901_3163_amd import deflan
    e = kappa_for("16x16x16x32")
    dims = tuple(e["dims"])
    ctx = deflan.Context(0)
    op = deflan.Operator(ctx, dims, torch.from_numpy(tiled_links(dims)).cuda(), e["kappa"], deflan.DL_G5M)
    net = deflan.Net(ctx, net_weights(args.net_seed, scale=1.0))
    B = torch.from_numpy(point_sources(dims)).cuda()
    out = {}
    for name, prec in (("fp32", deflan.DL_FP32), ("bf16", deflan.DL_BF16)):
        net.apply(op, B, prec=prec)
        torch.cuda.synchronize()
        t0 = time.time()
        for _ in range(args.reps):
            net.apply(op, B, prec=prec)
        torch.cuda.synchronize()
        out[name] = round((time.time() - t0) / args.reps * 1e3, 3)
        log(f"net forward {name}: {out[name]} ms per call (12 fields, including the host-side copies)")
    print(json.dumps(dict(kernel="learned-guess forward pass", dims=list(dims), nrhs=12, reps=args.reps,
                          ms_per_call=out)))
    net.close()
    op.close()
    ctx.close()


def drop_sweep(args):
    """The residual drop that ends an inner cycle of batched BF16 D-CG, from the projection-only
    start: the 4 held-out fields of the learned-guess workload (16^3x32, kappa tuned on field 10),
    Lan-DR(m,k) on M^dag M for a Gaussian first rhs (kept-vector re-orthogonalisation,
    eigenvectors lowered to FP32), then per field and drop one 64-rhs batched solve (BF16
    storage, FP32-eigenvector projection, reliable updates every 8 iterations) after a warm-up,
    the faster of two timed solves kept.  Prints one JSON line."""
    import torch
    from lattice_inputs import gaussian_spinor, gaussian_spinors_device, su3_links
    from paper_0901_3163_amd import deflan
    e = kappa_for("16x16x16x32/seed10")
    dims, kappa, tol = tuple(e["dims"]), e["kappa"], args.tol
    ctx = deflan.Context(0)
    drops = (1e-3, 1e-4, 3e-5, 1e-5, 3e-6, 1e-6)
    res = {f"{d:g}": dict(ms_per_field=[], iters_per_rhs=[], all_rhs_converged=True) for d in drops}
    for seed in (20, 21, 22, 23):
        U = torch.from_numpy(su3_links(dims, seed, e["eps"])).cuda()
        op = deflan.Operator(ctx, dims, U, kappa, deflan.DL_MDAGM)
        del U
        b1 = torch.from_numpy(gaussian_spinor(dims, 1000 + seed)).cuda()
        _, eig, _ = op.solve_first(b1, args.m, args.k, tol, reorth=deflan.DL_REORTH_KEPT)
        eig.lower(deflan.DL_FP32)
        B = gaussian_spinors_device(dims, 60000 + seed, args.test_rhs)
        kw = dict(storage=deflan.DL_BF16, batched=1, eig_storage=deflan.DL_FP32, reliable_every=8)
        op.solve_next(B, eig, tol, **kw)  # warm-up (tuning)
        for d in drops:
            ts = []
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.time()
                _, sts, rc = op.solve_next(B, eig, tol, inner_drop=d, **kw)
                torch.cuda.synchronize()
                ts.append(time.time() - t0)
            r = res[f"{d:g}"]
            r["ms_per_field"].append(round(1e3 * min(ts), 1))
            r["iters_per_rhs"].append(float(np.mean([s["iters"] for s in sts])))
            r["all_rhs_converged"] &= bool(rc == deflan.DL_OK and all(s["relres"] <= tol for s in sts))
            log(f"drop sweep: field {seed} drop {d:g}: {1e3 * min(ts):.1f} ms, "
                f"{np.mean([s['iters'] for s in sts]):.1f} iterations per rhs")
        eig.close()
        op.close()
    for r in res.values():
        r["rhs_per_s"] = round(4 * args.test_rhs / (sum(r["ms_per_field"]) / 1e3), 2)
    print(json.dumps(dict(workload=(f"16^3x32 Wilson (kappa {kappa:.6f}), held-out fields 20-23, Lan-DR({args.m},"
                                    f"{args.k}) on M^dag M, batched BF16 D-CG from the projection-only start for "
                                    f"{args.test_rhs} Gaussian rhs per field, tol {tol:g}"),
                          drops=res)))


def evenodd_study(args):
    """The even-odd (Schur complement) form against the whole-lattice system on held-out field 20
    of the learned-guess workload (16^3x32, kappa tuned on field 10): Lan-DR(m,k) for a Gaussian
    first rhs, then D-CG for 64 Gaussian rhs by plain FP64 (8 of them, one at a time) and by the
    batched BF16 path (all 64 together, FP32-rounded eigenvectors).  The even-odd runs include
    preparing bhat and reconstructing the whole solution; every solution is judged by its
    whole-lattice FP64 residual.  Prints one JSON line."""
    import torch
    from lattice_inputs import gaussian_spinor, gaussian_spinors_device, su3_links
    from paper_0901_3163_amd import deflan
    reorth = deflan.DL_REORTH_KEPT if args.reorth == "kept" else deflan.DL_REORTH_FULL
    os.environ.setdefault("DEFLAN_VERBOSE", "1")
    e = kappa_for("16x16x16x32/seed10")
    dims, kappa, tol = tuple(e["dims"]), e["kappa"], args.tol
    ctx = deflan.Context(0)
    U = torch.from_numpy(su3_links(dims, 20, e["eps"])).cuda()
    full = deflan.Operator(ctx, dims, U, kappa, deflan.DL_MDAGM)
    half = deflan.Operator(ctx, dims, U, kappa, deflan.DL_MDAGM | deflan.DL_EVEN_ODD)
    b1 = torch.from_numpy(gaussian_spinor(dims, 1020)).cuda()
    B = gaussian_spinors_device(dims, 60000, args.test_rhs)
    nb = torch.linalg.vector_norm(B.reshape(B.shape[0], -1), dim=1)
    out = dict(workload=(f"16^3x32 Wilson, held-out field 20 (kappa {kappa:.7f}), Lan-DR({args.m},{args.k}) on "
                         f"M^dag M then D-CG for {args.test_rhs} Gaussian rhs, tol {tol:g} on the whole-lattice "
                         "residual"), runs={})

    def whole_relres(X):
        nr = X.shape[0]
        R = B[:nr] - full.apply_batched(deflan.DL_APPLY_M, deflan.DL_FP64, X)
        return (torch.linalg.vector_norm(R.reshape(nr, -1), dim=1) / nb[:nr]).cpu().numpy()

    for name, op in (("whole", full), ("even_odd", half)):
        t0 = time.time()
        if op is half:
            bh = op.eo_prepare(b1)
            tol1 = tol * float(torch.linalg.vector_norm(b1)) / float(torch.linalg.vector_norm(bh))
            _, eig, st1 = op.solve_first(bh, args.m, args.k, tol1, reorth=reorth)
        else:
            _, eig, st1 = op.solve_first(b1, args.m, args.k, tol, reorth=reorth)
        eig.lower(deflan.DL_FP32)
        torch.cuda.synchronize()
        t_first = time.time() - t0
        res = dict(first_rhs=dict(mvp=st1["mvp"], mvp_lin=st1["mvp_lin"], seconds=round(t_first, 2),
                                  stop_rule=st1["stop_rule"]))
        log(f"evenodd {name}: first rhs {st1['mvp']} MVPs, {t_first:.1f}s")
        op.tune_wilson(deflan.DL_BF16, args.test_rhs, reps=3)
        for path, kw, nr in (("plain_fp64", dict(), args.plain_rhs),
                             ("batched_bf16", dict(storage=deflan.DL_BF16, batched=1, eig_storage=deflan.DL_FP32),
                              args.test_rhs)):
            Bs = B[:nr]
            for rep in range(2):  # the first pass warms up (launch shapes, buffers)
                torch.cuda.synchronize()
                t0 = time.time()
                if op is half:
                    Bh = torch.stack([op.eo_prepare(Bs[i]) for i in range(nr)])
                    nbh = torch.linalg.vector_norm(Bh.reshape(nr, -1), dim=1)
                    # the even system's tol that gives the whole-lattice tol (||r|| is the same)
                    tole = tol * float((nb[:nr] / nbh).min())
                    Xe, sts, rc = op.solve_next(Bh, eig, tole, **kw)
                    X = torch.stack([op.eo_reconstruct(Bs[i], Xe[i]) for i in range(nr)])
                else:
                    X, sts, rc = op.solve_next(Bs, eig, tol, **kw)
                torch.cuda.synchronize()
                dt = time.time() - t0
            rr = whole_relres(X)
            res[path] = dict(value=round(nr / dt, 3), unit="RHS/s", rhs=nr, iters_per_rhs=float(np.mean([s_["iters"] for s_ in sts])),
                             mvp_per_rhs=float(np.mean([s_["mvp"] for s_ in sts])),
                             max_whole_relres=float(rr.max()), all_converged=bool(rc == 0 and rr.max() <= tol * 1.0001))
            log(f"evenodd {name} {path}: {nr / dt:.2f} RHS/s, {res[path]['iters_per_rhs']:.0f} iterations per rhs, "
                f"whole-lattice relres {rr.max():.2e}")
        ms, by = op.bench_wilson(deflan.DL_APPLY_M, deflan.DL_BF16, args.test_rhs, 10)
        res["stencil_bf16_nrhs64"] = dict(avg_us=round(ms * 1e3, 1), bytes_per_launch=by,
                                         GBps=round(by / (ms * 1e-3) / 1e9, 1))
        out["runs"][name] = res
        eig.close()
    w, h = out["runs"]["whole"], out["runs"]["even_odd"]
    out["speedup_even_odd"] = {p_: round(h[p_]["value"] / w[p_]["value"], 3) for p_ in ("plain_fp64", "batched_bf16")}
    print(json.dumps(out), flush=True)
    half.close()
    full.close()
    ctx.close()


def window_sweep(args):
    """The batched D-MinRes of the benchmark workload in its fused short-recurrence form
    (minres_window < 0) and windowed with W = 8, 16, 32, 64: BF16 storage with the
    BF16-contracted projection, and FP32 storage with FP64 eigenvectors; projection-only
    starts, reps timed solves of the 12 point sources each.  Prints one JSON line."""
    import torch
    from lattice_inputs import gaussian_spinor, su3_links
    from paper_0901_3163_amd import deflan
    e = kappa_for("16x16x16x32")
    dims = tuple(e["dims"])
    ctx = deflan.Context(0)
    op = deflan.Operator(ctx, dims, torch.from_numpy(su3_links(dims, e["seed"], e["eps"])).cuda(), e["kappa"],
                         deflan.DL_G5M)
    _, eig, _ = op.solve_first(torch.from_numpy(gaussian_spinor(dims, 200)).cuda(), args.m, args.k, args.tol)
    eig.lower(deflan.DL_BF16)
    B = torch.from_numpy(point_sources(dims)).cuda()
    out = dict(workload=f"16^3x32 Wilson near-critical (kappa {e['kappa']:.7f}), 12 point sources, tol {args.tol:g}",
               reps=args.reps, runs={})
    for name, stg, est in (("bf16", deflan.DL_BF16, deflan.DL_BF16), ("fp32", deflan.DL_FP32, deflan.DL_FP64)):
        for win in (-1, 8, 16, 32, 64):
            kw = dict(storage=stg, batched=1, eig_storage=est, minres_window=win)
            op.solve_next(B, eig, args.tol, **kw)  # warm-up (tuning)
            torch.cuda.synchronize()
            t0 = time.time()
            for _ in range(args.reps):
                _, sts, rc = op.solve_next(B, eig, args.tol, **kw)
            torch.cuda.synchronize()
            dt = (time.time() - t0) / args.reps
            key = f"{name}/{'fused' if win < 0 else f'W{win}'}"
            out["runs"][key] = dict(value=round(12 / dt, 2), unit="RHS/s",
                                    iters_per_rhs=round(float(np.mean([s["iters"] for s in sts])), 1),
                                    max_relres=max(s["relres"] for s in sts), rc=rc)
            log(f"window sweep {key}: {12 / dt:.2f} RHS/s, {out['runs'][key]['iters_per_rhs']} iterations per rhs")
    print(json.dumps(out))
    eig.close()
    op.close()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--pairs", type=int, default=256, help="training pairs per training field")
    ap.add_argument("--test-rhs", type=int, default=64, help="right-hand sides per held-out field")
    ap.add_argument("--plain-rhs", type=int, default=8, help="rhs per held-out field of the plain FP64 baseline")
    ap.add_argument("--epochs", type=int, default=2, help="passes of the network training over the fields")
    ap.add_argument("--reorth", choices=("full", "kept"), default="kept",
                    help="re-orthogonalisation of the first-rhs Lan-DR runs")
    ap.add_argument("--no-c2", action="store_true", help="skip the plain-method (C2) extra keys")
    ap.add_argument("--c2-steps", type=int, default=3, help="timed steps of the C2 extra keys")
    ap.add_argument("--plain-steps", type=int, default=1, help="timed steps of the plain FP64 baseline")
    ap.add_argument("--m", type=int, default=120)
    ap.add_argument("--k", type=int, default=60)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-sweep", action="store_true", help="skip the Dslash bandwidth sweep")
    ap.add_argument("--kappa", type=float, default=None, help="override the stored kappa (exploration only)")
    ap.add_argument("--inner-drop", type=float, default=None,
                    help="headline: residual drop per inner cycle of the batched D-CG (default: the library's)")
    ap.add_argument("--kernel-only", action="store_true", help="run only the dominant kernel + a copy (profiling)")
    ap.add_argument("--ko-lattice", default=None, help="--kernel-only on this lattice (e.g. 32x32x32x64) instead")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--train-rhs", type=int, default=24, help="training pairs of the learned guess (0: no net)")
    ap.add_argument("--train-steps", type=int, default=100, help="Adam steps per field and pass")
    ap.add_argument("--train-batch", type=int, default=6)
    ap.add_argument("--train-lr", type=float, default=3e-3)
    ap.add_argument("--net-seed", type=int, default=7)
    ap.add_argument("--ablation-steps", type=int, default=1)
    ap.add_argument("--storage", choices=("fp32", "bf16"), default="bf16",
                    help="Krylov-vector storage of the timed fast path")
    ap.add_argument("--eig-storage", choices=("fp64", "fp32", "bf16"), default="bf16",
                    help="eigenvectors the projection of the timed fast path reads")
    ap.add_argument("--net-prec", choices=("fp32", "bf16"), default="bf16",
                    help="inference precision of the learned guess on the timed fast path")
    ap.add_argument("--multi", action="store_true", help="the uneven multi-lattice batch instead (own JSON line)")
    ap.add_argument("--multi-storage", choices=("fp32", "bf16"), default="bf16")
    ap.add_argument("--multi-critical", action="store_true",
                    help="--multi at near-critical kappa per lattice (links seed 0)")
    ap.add_argument("--precision", action="store_true",
                    help="the 24^3x48 precision study instead (own JSON line)")
    ap.add_argument("--prec-m", type=int, default=200)
    ap.add_argument("--prec-k", type=int, default=100)
    ap.add_argument("--no-proj-sweep", action="store_true", help="skip the deflation-contraction sweep")
    ap.add_argument("--proj-only", action="store_true", help="run only the deflation contraction (profiling)")
    ap.add_argument("--ksweep", action="store_true",
                    help="the k-sweep on a 20^3x32 field instead (own JSON line)")
    ap.add_argument("--net-only", action="store_true", help="run only the network's forward pass (profiling)")
    ap.add_argument("--learned", action="store_true",
                    help="the learned-guess study across training and held-out fields instead (own JSON line)")
    ap.add_argument("--window-sweep", action="store_true",
                    help="the D-MinRes window sweep on the benchmark workload instead (own JSON line)")
    ap.add_argument("--tune-report", action="store_true",
                    help="the autotuner's choices at the paths' sizes (own JSON line)")
    ap.add_argument("--evenodd", action="store_true",
                    help="the even-odd (Schur) form against the whole lattice on a held-out field instead")
    ap.add_argument("--drop-sweep", action="store_true",
                    help="the inner-cycle residual drop of batched BF16 D-CG on the held-out fields (own JSON line)")
    ap.add_argument("--learned-pairs", type=int, default=256)
    ap.add_argument("--learned-test", type=int, default=64)
    ap.add_argument("--learned-epochs", type=int, default=2)
    ap.add_argument("--learned-steps", type=int, default=100)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path is not sharded across GPUs.",
              file=sys.stderr)
        sys.exit(2)

    if args.kernel_only:
        return kernel_only(args)
    if args.multi:
        return multi_lattice(args)
    if args.precision:
        return precision_study(args)
    if args.proj_only:
        return projection_only(args)
    if args.learned:
        return learned_study(args)
    if args.net_only:
        return net_only(args)
    if args.ksweep:
        return ksweep_study(args)
    if args.window_sweep:
        return window_sweep(args)
    if args.evenodd:
        return evenodd_study(args)
    if args.drop_sweep:
        return drop_sweep(args)
    if args.tune_report:
        return tune_report(args)
    os.environ.setdefault("DEFLAN_VERBOSE", "1")  # per-cycle progress lines from the library
    return c5_headline(args)


def cpu_baseline_dcg(dims, kappa, seed, b_host, iters_per_rhs, k):
    """Oracle D-CG on the host cores for a bounded sample: the Galerkin projection over k seeded
    orthonormal vectors and 60 CGLS iterations on one right-hand side of the held-out workload
    (numpy vectors, the OpenMP C Wilson matrix), scaled to the GPU's iterations per rhs."""
    from lattice_inputs import su3_links
    from oracle import cwilson, deflated, krylov
    cores = len(os.sched_getaffinity(0))
    op = cwilson.CWilson(su3_links(dims, seed), dims, kappa)
    n = op.n
    rng = np.random.default_rng(7)
    Y, _ = np.linalg.qr(rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k)))
    b = np.ascontiguousarray(b_host.ravel())
    t0 = time.time()
    H = deflated.projection_matrix(op.MdagM, Y)  # once per handle, not per rhs
    t_h = time.time() - t0
    nit = 60
    t0 = time.time()
    x0 = deflated.galerkin_projection(Y, H, op.Mdag(b))
    t_proj = time.time() - t0
    t0 = time.time()
    krylov.cgls(op.M, op.Mdag, b, x0=x0, tol=0.0, maxiter=nit)
    t_it = (time.time() - t0) / nit
    per_rhs = t_proj + iters_per_rhs * t_it
    return dict(value=round(1.0 / per_rhs, 5), unit="RHS/s", cores=cores, kind="oracle",
                sample=(f"oracle D-CG (numpy vectors, OpenMP C Wilson matrix) on {'x'.join(map(str, dims))}, held-out "
                        f"field {seed}: Galerkin projection of M^dag b over {k} seeded orthonormal vectors "
                        f"({t_proj:.2f}s) + {nit} CGLS iterations ({t_it * 1e3:.1f} ms/iter) on one right-hand side "
                        f"of the workload; per-rhs time = projection + {iters_per_rhs:.0f} iterations (the plain FP64 "
                        f"GPU run's mean per rhs); H = Y^H A Y setup ({t_h:.1f}s) excluded like the GPU's"),
                seconds_per_rhs=round(per_rhs, 3))


def c5_headline(args):
    """The learned-guess configuration, on which the metric is quoted: 16^3x32 Wilson, one kappa
    (tuned on links seed 10 to min|lambda(gamma5 M)| = 1e-3) for training fields 10-17 and
    held-out fields 20-23.  Setup (untimed, reported): per field Lan-DR(m,k) on M^dag M for a
    Gaussian first rhs (eigenvectors lowered to FP32); per training field 256 Gaussian (b, x) pairs
    solved to tol by the batched path; the network trained on them in FP32 on the GPU (Adam), with
    the loss on the error the D-CG projection leaves.  One timed step: D-CG for the 4 held-out
    fields x 64 Gaussian rhs, each field's 64 rhs in one batch: BF16 Krylov vectors and stencil
    spinors (FP32 arithmetic and links), FP64 true residuals and solutions, the Galerkin projection
    over the field's FP32-rounded eigenvectors, and the learned guess (BF16 inference of its middle
    layer); every rhs verified by its FP64 true residual <= tol.  Baseline: plain FP64 D-CG one rhs
    at a time over the same FP64 eigenvectors and right-hand sides."""
    import torch
    from lattice_inputs import gaussian_spinor, gaussian_spinors_device, net_weights, su3_links
    from paper_0901_3163_amd import deflan
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    e = kappa_for("16x16x16x32/seed10")
    dims, kappa, tol = tuple(e["dims"]), e["kappa"], args.tol
    V = int(np.prod(dims))
    m, k = args.m, args.k
    reorth = deflan.DL_REORTH_KEPT if args.reorth == "kept" else deflan.DL_REORTH_FULL
    npair, ntest, bs = args.pairs, args.test_rhs, 64
    ctx = deflan.Context(0)
    BF, F32, F64 = deflan.DL_BF16, deflan.DL_FP32, deflan.DL_FP64

    def field(seed):
        U = torch.from_numpy(su3_links(dims, seed, e["eps"])).cuda()
        op = deflan.Operator(ctx, dims, U, kappa, deflan.DL_MDAGM)
        del U
        t0 = time.time()
        b1 = torch.from_numpy(gaussian_spinor(dims, 1000 + seed)).cuda()
        _, eig, st1 = op.solve_first(b1, m, k, tol, reorth=reorth)
        eig.lower(F32)
        torch.cuda.synchronize()
        dt = time.time() - t0
        log(f"field {seed}: Lan-DR({m},{k}) {st1['mvp']} MVPs ({st1['mvp_lin']} to tol), {dt:.1f}s, "
            f"rule {st1['stop_rule']}")
        return op, eig, dict(seed=seed, mvp=st1["mvp"], mvp_lin=st1["mvp_lin"], seconds=round(dt, 2),
                             relres=st1["relres"], stop_rule=st1["stop_rule"])

    def solve(op, eig, B, **kw):
        X = torch.empty_like(B)
        its, kept, ok = [], [], True
        for i in range(0, B.shape[0], bs):
            Xi, sts, rc = op.solve_next(B[i:i + bs], eig, tol, batched=1, inner_drop=args.inner_drop, **kw)
            X[i:i + bs] = Xi
            its += [s["iters"] for s in sts]
            kept += [s["guess"] for s in sts]
            ok &= rc == deflan.DL_OK and all(s["relres"] <= tol for s in sts)
        return X, its, kept, ok

    # ---- setup: training fields, pairs, network ----
    t_setup = time.time()
    train, first = [], []
    t_pairs = 0.0
    pair_iters = []
    for seed in range(10, 18):
        op, eig, info = field(seed)
        first.append(info)
        B = gaussian_spinors_device(dims, 20000 + 1000 * seed, npair)
        t0 = time.time()
        X, its, _, ok = solve(op, eig, B, storage=BF, eig_storage=F32)
        torch.cuda.synchronize()
        t_pairs += time.time() - t0
        pair_iters += its
        assert ok, f"training pairs of field {seed} did not reach tol"
        train.append((op, eig, B, X))
        log(f"field {seed}: {npair} training pairs in {time.time() - t0:.1f}s, {np.mean(its):.0f} iterations per rhs")
    net = deflan.Net(ctx, net_weights(args.net_seed))
    t0 = time.time()
    losses = []
    for ep in range(args.epochs):
        for op, eig, B, X in train:
            net.set_projection(eig)
            losses += list(net.train(op, B, X, batch=args.train_batch, steps=args.train_steps, lr=args.train_lr))
    net.set_projection(None)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    log(f"network: {len(losses)} Adam steps in {t_train:.1f}s, loss {losses[0]:.4f} -> {np.mean(losses[-20:]):.4f}")
    for op, eig, B, X in train:
        eig.close()
        op.close()
    del train, B, X
    torch.cuda.empty_cache()
    held = []
    for seed in range(20, 24):
        op, eig, info = field(seed)
        first.append(info)
        # stencil launch shapes of every configuration timed below, tuned here (untimed)
        for prec, nr in ((BF, ntest), (F32, ntest), (F64, ntest), (F64, 1)):
            op.tune_wilson(prec, nr, reps=3)
        held.append((op, eig, gaussian_spinors_device(dims, 40000 + 1000 * seed, ntest), seed))
    # and the projection's contraction shapes (the plain baseline's one-column kernels need none)
    pretune_projection(ctx, deflan, V * 12, k, ntest)
    setup_s = time.time() - t_setup

    fast_kw = dict(storage=BF, eig_storage=F32, net=net, net_prec=BF)

    def step(**kw):
        its, kept, ok = [], [], True
        for op, eig, B, _ in held:
            _, it, kp, o = solve(op, eig, B, **kw)
            its += it
            kept += kp
            ok &= o
        return its, kept, ok

    for w in range(args.warmup):
        its, _, _ = step(**fast_kw)
        log(f"warmup {w}: {np.mean(its):.1f} iterations per rhs")
    torch.cuda.synchronize()
    ctx.timing(True)
    t0 = time.time()
    all_ok, iters, kept = True, [], []
    for s_ in range(args.steps):
        its, kp, ok = step(**fast_kw)
        all_ok &= ok
        iters += its
        kept += kp
        log(f"step {s_}: {np.mean(its):.1f} iterations per rhs, all converged {ok}")
    torch.cuda.synchronize()
    dt = time.time() - t0
    n_w, ms_w, by_w = ctx.kernel_time("wilson")
    ctx.timing(False)
    nrhs_step = len(held) * ntest
    value = nrhs_step * args.steps / dt
    log(f"fast path: {value:.2f} RHS/s")

    # ---- ablation: each factor on one pass over the held-out set ----
    ablation = {}
    for name, kw in (("bf16+proj_fp32", dict(storage=BF, eig_storage=F32)),
                     ("bf16+proj_fp64", dict(storage=BF, eig_storage=F64)),
                     ("fp32+proj_fp32", dict(storage=F32, eig_storage=F32)),
                     ("fp32+proj_fp32+net", dict(storage=F32, eig_storage=F32, net=net, net_prec=F32)),
                     ("bf16+proj_fp32+net_fp32", dict(storage=BF, eig_storage=F32, net=net, net_prec=F32))):
        torch.cuda.synchronize()
        t1 = time.time()
        its, kp, ok = step(**kw)
        torch.cuda.synchronize()
        d1 = time.time() - t1
        ablation[name] = dict(value=round(nrhs_step / d1, 3), unit="RHS/s", iters_per_rhs=float(np.mean(its)),
                              all_rhs_converged=bool(ok), guess_kept=float(np.mean(kp)) if "net" in kw else None)
        log(f"ablation {name}: {nrhs_step / d1:.2f} RHS/s, {np.mean(its):.1f} iterations per rhs")
    proj_only = ablation["bf16+proj_fp32"]

    # ---- baseline: plain FP64 D-CG, one rhs at a time, same eigenvectors (FP64) and rhs ----
    log("plain FP64 D-CG baseline")
    op0, eig0, B0, _ = held[0]
    op0.solve_next(B0[:1], eig0, tol)  # warm-up
    torch.cuda.synchronize()
    t1 = time.time()
    its64, ok64, n64 = [], True, 0
    for op, eig, B, _ in held:
        _, sts, rc = op.solve_next(B[:args.plain_rhs], eig, tol)
        its64 += [s_["iters"] for s_ in sts]
        ok64 &= rc == deflan.DL_OK and all(s_["relres"] <= tol for s_ in sts)
        n64 += args.plain_rhs
    torch.cuda.synchronize()
    d64 = time.time() - t1
    plain_value = n64 / d64
    log(f"plain FP64 D-CG {plain_value:.2f} RHS/s; fast path {value / plain_value:.2f}x")

    achieved = by_w / (ms_w * 1e-3) / 1e9 if ms_w > 0 else 0.0
    bpl = by_w / max(n_w, 1)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic_from_profiles(dims, "bf16", ntest),
                    kernel=("Wilson stencil (M and M^dag of D-CG), BF16 spinors, FP32 links and arithmetic, batched "
                            f"over the {ntest} rhs of a held-out field (tuned launch shape)"),
                    launches=n_w, avg_us=round(ms_w / max(n_w, 1) * 1e3, 2), bytes_per_launch=round(bpl),
                    note=(f"algorithmic bytes per launch: links once (288 B/site FP32) + input and output spinor "
                          f"per active rhs (96 B/site BF16); {round(bpl / 1e6)} MB on average per launch "
                          f"({V * (288 + 96 * ntest) / 1e6:.0f} MB with all {ntest} rhs active), above the 256 MB "
                          "Infinity Cache"))
    result = dict(metric=METRIC, value=round(value, 3), unit="RHS/s", n_gpus=1, steps=args.steps,
                  warmup=args.warmup, ms_per_step=round(dt / args.steps * 1e3, 2), higher_is_better=True,
                  scaling="weak", vs_baseline=None, dtype="bf16/f32+f64",
                  data="synthetic (seeded SU(3) gauge fields and Gaussian right-hand sides)",
                  config=dict(workload=(f"learned-guess held-out set: 16^3x32 Wilson, kappa {kappa:.7f} tuned on "
                                        f"links seed 10 (min|lambda(gamma5 M)| {e['min_abs_eig']:.2e}), network "
                                        f"trained on {8 * npair} (b, x) pairs from D-CG on fields 10-17, tested on "
                                        f"held-out fields 20-23 x {ntest} Gaussian rhs; Lan-DR({m},{k}) on M^dag M "
                                        f"per field, then D-CG from net(b) + projection, tol {tol:g}"),
                              lattice=list(dims), kappa=kappa, training_fields=list(range(10, 18)),
                              held_out_fields=list(range(20, 24)), rhs_per_field=ntest, m=m, k=k,
                              reorth=args.reorth,
                              path=("batched D-CG (CG on M^dag M x = M^dag b), the 64 rhs of a field in one batch: "
                                    "BF16 Krylov vectors and Wilson apply (FP32 arithmetic and links), FP64 "
                                    "reliable updates and true residuals, FP64 solution, Galerkin projection over "
                                    "the FP32-rounded eigenvectors (FP64 arithmetic), learned initial guess (BF16 "
                                    "matrix-core inference of the 16->16 layer; net(b) + projection, kept per rhs "
                                    "when its residual is smaller)")),
                  all_rhs_converged=bool(all_ok), iters_per_rhs=float(np.mean(iters)),
                  guess_kept_per_rhs=float(np.mean(kept)),
                  learned_guess=dict(training_pairs=8 * npair, pair_seconds=round(t_pairs, 2),
                                     pair_iters_per_rhs=float(np.mean(pair_iters)), epochs=args.epochs,
                                     steps_per_field=args.train_steps, batch=args.train_batch, lr=args.train_lr,
                                     adam_steps=len(losses), train_seconds=round(t_train, 2),
                                     loss_first=round(float(losses[0]), 5),
                                     loss_last20=round(float(np.mean(losses[-20:])), 5),
                                     loss="mean ||M d'||^2 / ||b||^2, d' = the error of net(b) left after the D-CG "
                                          "Galerkin projection over the field's eigenvectors",
                                     iters_saved_per_rhs=round(proj_only["iters_per_rhs"] - float(np.mean(iters)), 2),
                                     rhs_per_s_vs_projection_only=round(value / proj_only["value"], 4)),
                  ablation=ablation,
                  plain_fp64=dict(value=round(plain_value, 3), unit="RHS/s", rhs=n64,
                                  all_rhs_converged=bool(ok64), iters_per_rhs=float(np.mean(its64)),
                                  path=f"D-CG FP64, one rhs after another (first {args.plain_rhs} rhs of each "
                                       "held-out field)"),
                  speedup_vs_plain_fp64=round(value / plain_value, 3),
                  first_rhs=first, setup_seconds=round(setup_s, 1),
                  roofline=roofline)
    if not args.no_sweep:
        result["dslash_sweep"] = dslash_sweep(ctx, deflan, [(24, 24, 24, 48), (32, 32, 32, 64)], reps=20)
        result["dslash_sweep"]["16x16x16x32/bf16/nrhs64"] = dslash_point(held[0][0], deflan, deflan.DL_BF16, ntest, 20)
        result["copy_ceiling"] = copy_ceiling(ctx)
    if not args.no_c2:
        result["c2"] = c2_workload(args, ctx, deflan)
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        op_h, _, B_h, seed_h = held[0]
        result["cpu_baseline"] = cpu_baseline_dcg(dims, kappa, seed_h, B_h[0].cpu().numpy(),
                                                  result["plain_fp64"]["iters_per_rhs"], k)
    for op, eig, B, _ in held:
        eig.close()
        op.close()
    net.close()
    ctx.close()
    print(json.dumps(result), flush=True)


def c2_workload(args, ctx, deflan):
    """The plain-method configuration (16^3x32 near-critical, min|lambda| ~ 1e-4, seed 0):
    MinRes-DR(m,k) on gamma5 M for a Gaussian first rhs, then the 12 spin-colour point sources
    by the batched BF16 D-MinRes (with a network trained on 24 point sources of the same field)
    and by plain FP64 D-MinRes one rhs at a time.  Returns a dict (extra keys of the benchmark
    line)."""
    import torch
    from lattice_inputs import gaussian_spinor, su3_links
    try:
        e = kappa_for("16x16x16x32")
    except KeyError:
        e = dict(dims=[16, 16, 16, 32], seed=0, eps=0.5, kappa=None)
    dims = tuple(e["dims"])
    kappa = args.kappa if args.kappa is not None else e["kappa"]
    if kappa is None:
        sys.exit("no kappa stored for 16x16x16x32: run `python -m oracle.kappa large`")
    V = int(np.prod(dims))
    log(f"C2 workload 16^3x32 kappa={kappa:.7f}: building operator")
    U = torch.from_numpy(su3_links(dims, e["seed"], e["eps"])).cuda()
    op = deflan.Operator(ctx, dims, U, kappa, deflan.DL_G5M)
    b1 = torch.from_numpy(gaussian_spinor(dims, 200)).cuda()
    log(f"first rhs: MinRes-DR({args.m},{args.k}), re-orthogonalisation {args.reorth}")
    t0 = time.time()
    x1, eig, st1 = op.solve_first(b1, args.m, args.k, args.tol,
                                  reorth=deflan.DL_REORTH_KEPT if args.reorth == "kept" else deflan.DL_REORTH_FULL)
    torch.cuda.synchronize()
    t_first = time.time() - t0
    log(f"first rhs done: {st1['mvp']} MVPs ({st1['mvp_lin']} at linear convergence), {t_first:.1f}s, "
        f"relres {st1['relres']:.2e}, rule {st1['stop_rule']}")
    B = torch.from_numpy(point_sources(dims)).cuda()
    nrhs = B.shape[0]

    # learned initial guess (setup, untimed): train the network on point sources at other
    # sites of the same field, solved by the mixed-precision batched path
    net, net_info = None, None
    if args.train_rhs > 0:
        net, net_info = train_guess(ctx, op, eig, deflan, dims, args)

    storage = {"fp32": deflan.DL_FP32, "bf16": deflan.DL_BF16}[args.storage]
    eig_storage = {"fp64": deflan.DL_FP64, "fp32": deflan.DL_FP32, "bf16": deflan.DL_BF16}[args.eig_storage]
    # lowered eigenvector copies (setup: k MVPs for the FP32 basis's Gram matrix); a BF16
    # handle serves FP32 as well
    t0 = time.time()
    lower_mvp = eig.lower(deflan.DL_BF16)
    torch.cuda.synchronize()
    lowering = dict(mvp=lower_mvp, seconds=round(time.time() - t0, 2))
    pretune_projection(ctx, deflan, V * 12, args.k, nrhs)

    net_prec = {"fp32": deflan.DL_FP32, "bf16": deflan.DL_BF16}[args.net_prec]

    def fast(use_net=True, st=None, eig_st=None, nprec=None):
        return op.solve_next(B, eig, args.tol, storage=storage if st is None else st, batched=1,
                             net=net if use_net else None,
                             eig_storage=eig_storage if eig_st is None else eig_st,
                             net_prec=net_prec if nprec is None else nprec)

    def plain():
        return op.solve_next(B, eig, args.tol)

    for w in range(1):
        X, sts, rc = fast()
        log(f"warmup {w} (batched FP32{' + learned guess' if net else ''}): iters {[s['iters'] for s in sts]}")
    torch.cuda.synchronize()
    ctx.timing(True)
    t0 = time.time()
    all_ok = True
    iters, kept = [], []
    for s in range(args.c2_steps):
        X, sts, rc = fast()
        all_ok &= all(st["relres"] <= args.tol for st in sts)
        iters += [st["iters"] for st in sts]
        kept += [st["guess"] for st in sts]
        log(f"step {s}: rc {rc}, max relres {max(st['relres'] for st in sts):.2e}")
    torch.cuda.synchronize()
    dt = time.time() - t0
    n_w, ms_w, by_w = ctx.kernel_time("wilson")
    ctx.timing(False)
    value = nrhs * args.c2_steps / dt
    # ablation: the batched path with each storage, with and without the learned guess
    ablation = {}
    if net is not None:
        net_info["guess_kept_per_rhs"] = float(np.mean(kept))
    E64, E32, E16 = deflan.DL_FP64, deflan.DL_FP32, deflan.DL_BF16
    N32, N16 = deflan.DL_FP32, deflan.DL_BF16
    for name, st_, use_net, est, npr in (("fp32", deflan.DL_FP32, False, E64, N32),
                                         ("bf16", deflan.DL_BF16, False, E64, N32),
                                         ("fp32+guess", deflan.DL_FP32, True, E64, N32),
                                         ("bf16+guess", deflan.DL_BF16, True, E64, N32),
                                         ("fp32+eig_fp32", deflan.DL_FP32, False, E32, N32),
                                         ("bf16+eig_bf16", deflan.DL_BF16, False, E16, N32),
                                         ("bf16+eig_bf16+guess", deflan.DL_BF16, True, E16, N32),
                                         ("bf16+eig_bf16+guess_bf16", deflan.DL_BF16, True, E16, N16)):
        if use_net and net is None:
            continue
        fast(use_net, st_, est, npr)
        torch.cuda.synchronize()
        t0 = time.time()
        for s in range(args.ablation_steps):
            Xm, stm, _ = fast(use_net, st_, est, npr)
        torch.cuda.synchronize()
        dtm = time.time() - t0
        ablation[name] = dict(value=round(nrhs * args.ablation_steps / dtm, 3), unit="RHS/s",
                              steps=args.ablation_steps,
                              all_rhs_converged=bool(all(st["relres"] <= args.tol for st in stm)),
                              iters_per_rhs=float(np.mean([st["iters"] for st in stm])),
                              max_relres=float(max(st["relres"] for st in stm)))
        log(f"ablation {name}: {ablation[name]['value']:.2f} RHS/s, iters {ablation[name]['iters_per_rhs']:.1f}")
    achieved = by_w / (ms_w * 1e-3) / 1e9
    sp_b = 96 if args.storage == "bf16" else 192
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic_from_profiles(dims, args.storage),
                    kernel=(f"Wilson stencil, gamma5 M, {args.storage.upper()} spinors, FP32 links and arithmetic, "
                            "batched over right-hand sides (tuned launch shape)"), launches=n_w,
                    avg_us=round(ms_w / max(n_w, 1) * 1e3, 2), bytes_per_launch=round(by_w / max(n_w, 1)),
                    note=(f"algorithmic bytes per launch: links once (288 B/site FP32) + input and output "
                          f"spinor per active rhs ({sp_b} B/site); the 16^3x32 working set is about the size of "
                          "the 256 MB Infinity Cache, see dslash_sweep for HBM-resident sizes"))
    # plain FP64 D-MinRes, one rhs after another: the baseline the fast path is compared with
    log("plain FP64 baseline")
    X64, st64, _ = plain()
    torch.cuda.synchronize()
    t0 = time.time()
    for s in range(args.plain_steps):
        X64, st64, _ = plain()
    torch.cuda.synchronize()
    dt64 = time.time() - t0
    plain_value = nrhs * args.plain_steps / dt64
    ok64 = all(st["relres"] <= args.tol for st in st64)
    log(f"fast {value:.2f} RHS/s, plain FP64 {plain_value:.2f} RHS/s")
    result = dict(value=round(value, 3), unit="RHS/s", steps=args.c2_steps,
                  ms_per_step=round(dt / args.c2_steps * 1e3, 2),
                  config=dict(workload=f"16^3x32 Wilson near-critical (kappa {kappa:.6f}), MinRes-DR({args.m},"
                                       f"{args.k}) on gamma5 M then D-MinRes on 12 point sources, tol "
                                       f"{args.tol:g}", lattice=list(dims), kappa=kappa, nrhs=nrhs,
                              m=args.m, k=args.k,
                              path=("batched D-MinRes (windowed: Lanczos vectors in a ring, solution formed "
                                    f"every 64 iterations), {args.storage.upper()} Krylov vectors and Wilson apply "
                                    "(FP32 arithmetic and links), FP64 residuals and solution, projection over "
                                    + {"fp64": "FP64 eigenvectors",
                                       "fp32": "FP32 eigenvectors (matrix-core contraction)",
                                       "bf16": "BF16-contracted, FP32-corrected eigenvectors (matrix cores)"}[
                                           args.eig_storage]
                                    + (f", learned initial guess ({args.net_prec.upper()} inference; net(b) + "
                                       "projection, kept per rhs when its residual is smaller)"
                                       if net is not None else ""))),
                  all_rhs_converged=bool(all_ok), iters_per_rhs=float(np.mean(iters)),
                  learned_guess=net_info, ablation_batched=ablation,
                  plain_fp64=dict(value=round(plain_value, 3), unit="RHS/s", steps=args.plain_steps,
                                  all_rhs_converged=bool(ok64),
                                  iters_per_rhs=float(np.mean([st["iters"] for st in st64])),
                                  path="D-MinRes FP64, one rhs after another"),
                  speedup_vs_plain_fp64=round(value / plain_value, 3),
                  eigenvector_lowering=lowering,
                  first_rhs=dict(mvp=st1["mvp"], mvp_lin=st1["mvp_lin"], seconds=round(t_first, 2),
                                 relres=st1["relres"], stop_rule=st1["stop_rule"], reorth=args.reorth,
                                 mvp_overhead=round(st1["mvp"] / max(st1["mvp_lin"], 1), 3)),
                  roofline=roofline)
    if net is not None:
        net.close()
    eig.close()
    op.close()
    return result

if __name__ == "__main__":
    main()
