"""Benchmark of the IDBF hot path on one MI355X.

One step = the whole hot path on the N = 2^20 FIO workload
(Phi = x xi + c(x)|xi|, c(x) = (2 + sin 2 pi x)/8, leaf 16, tol 1e-6,
oversampling t = 2): construction (FP64 IDs on the GPU), then applies of the
factors with every input resident in HBM:

  complex64   1 RHS (VALU), 256 and 1024 RHS (FP32 MFMA)
  BF16 split  256 and 1024 RHS (BF16 hi/lo MFMA products, FP32 accumulation)
  complex128  1, 256 and 1024 RHS (the plain FP64 form, VALU)

Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] ...
    python bench.py --only learned      # the learned proposal at full scale
                                        # (2000 training constructions, 200 held out)

value = algorithmic GB/s of the complex64 1-RHS apply (factor entries + ID
records + x and y once), averaged over the timed steps; every other apply is
reported beside it with its rate, its relative error against the complex128
apply of the same factors on 8 probe vectors, and its speedup over the
complex128 apply of the same right-hand-side count.  "roofline" is computed
live from HIP events the library records around every launch, for the kernel
that takes the largest share of a step.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import tempfile
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1809_10573_amd import inputs as I  # noqa: E402

METRIC = "IDBF apply GB/s+GFLOP/s & construct ms, N=2^20, vs plain FP64 at rel.err 1e-6"
HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK = 78.6e12
FP64_MFMA_PEAK = 78.6e12
FP32_MFMA_PEAK = 157.3e12
BF16_MFMA_PEAK = 2500e12

WORKLOAD = dict(N=1 << 20, leaf=16, tol=1e-6, oversample=2, a=1.0, freq=1.0, c0=2.0, cdiv=8.0)


def _cpu_baseline(timeout_s: int = 400) -> dict | None:
    """The oracle on the host cores, before anything initializes the GPU, on
    the N = 2^16 member of the same FIO kernel (leaf 16, tol 1e-6, t = 2):
    its construction on all host cores (one process per core over the
    independent IDs of each level), its complex128 apply on one thread, and
    its construction on one thread at N = 2^13 (the single-thread build at
    N = 2^16 takes minutes)."""
    code = r"""
import json, os, sys, time
sys.path.insert(0, %r)
import numpy as np
import oracle
from paper_1809_10573_amd import inputs as I
ph = I.fio_phase(1.0, 1.0)
cores = max(1, min(16, os.cpu_count() or 1))
N, leaf, tol, t = 1 << 16, 16, 1e-6, 2
X, O = I.uniform_grid(N)
t0 = time.perf_counter()
F = oracle.build(ph, X, O, leaf, tol, oversample=t, workers=cores)
build_all = time.perf_counter() - t0
g = I.gaussian_vectors(N, None, 4)
reps = 3
t0 = time.perf_counter()
for _ in range(reps):
    y = oracle.apply(F, g)
apply_s = (time.perf_counter() - t0) / reps
nnz = F.nnz()
n_ids = sum(len(F.U[k]) + len(F.V[k]) for k in F.U)
Ns = 1 << 13
Xs, Os = I.uniform_grid(Ns)
t0 = time.perf_counter()
Fs = oracle.build(ph, Xs, Os, leaf, tol, oversample=t)
build_1 = time.perf_counter() - t0
n_ids_s = sum(len(Fs.U[k]) + len(Fs.V[k]) for k in Fs.U)
print(json.dumps(dict(N=N, nnz=nnz, n_ids=n_ids, build_all_s=build_all, cores=cores, apply_s=apply_s,
                      gbs=(nnz * 16 + 8 * n_ids + 2 * N * 16) / apply_s / 1e9, Ns=Ns, build_1_s=build_1,
                      n_ids_s=n_ids_s, cpu_count=os.cpu_count())))
""" % ROOT
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    try:
        res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                             timeout=timeout_s, env=env)
    except subprocess.TimeoutExpired:
        return None
    if res.returncode != 0:
        print(res.stderr[-2000:], file=sys.stderr)
        return None
    r = json.loads(res.stdout.strip().splitlines()[-1])
    return {"value": r["gbs"], "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle FP64 (complex128) apply of its own N=2^16 factorization of the same FIO "
                       f"kernel (leaf 16, tol 1e-6, t=2; {r['nnz']} stored entries), 1 thread: "
                       f"{r['apply_s'] * 1e3:.0f} ms per apply"),
            "construct_s_all_cores": r["build_all_s"], "construct_cores": r["cores"],
            "host_cpu_count": r["cpu_count"],
            "construct_ids_per_s_all_cores": r["n_ids"] / r["build_all_s"],
            "construct_s_1thread_n2p13": r["build_1_s"],
            "construct_ids_per_s_1thread": r["n_ids_s"] / r["build_1_s"]}


def _batched(B, torch, dev, stream) -> dict:
    """The many-instance workload (64 instances, N = 2^12..2^18, DFT and FIO
    family members, nrhs in {1, 16, 64}, complex64 apply): one-by-one versus
    idbf_construct_batched / idbf_apply_batched after a warm-up; the
    constructions are the fastest of three wall-clock runs (see
    timed_construct), the applies one event-timed run each."""
    work = I.batched_workload()
    Xs, Os = [], []
    for w in work:
        X, O = I.uniform_grid(w["N"])
        Xs.append(torch.as_tensor(X, device=dev))
        Os.append(torch.as_tensor(O, device=dev))
    gen = torch.Generator(device=dev).manual_seed(6)
    xs = [torch.randn(w["N"], w["nrhs"], dtype=torch.complex64, device=dev, generator=gen).squeeze(1)
          * np.sqrt(2.0) for w in work]
    xs = [x.contiguous() for x in xs]
    ys = [torch.empty_like(x) for x in xs]
    args = ([w["phase"] for w in work], Xs, Os, [w["tol"] for w in work], [w["leaf"] for w in work])

    def timed_apply(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()  # warm-up
        torch.cuda.synchronize()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    def timed_construct(fn, keep):
        """Wall time of fn() (a list of factorizations) over three runs: the
        fastest, every sample, and the last run's factorizations if keep.
        The fastest: on the GPU machines single runs of either path sometimes
        stall on the host for 0.5-3 s with the GPU idle (kernel times
        unchanged), which a median of three does not always exclude."""
        times, facs = [], None
        for rep in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            facs = fn()
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
            if rep < 2 or not keep:
                for f in facs:
                    f.close()
                facs = None
        return float(min(times)), [round(t, 1) for t in times], facs

    # one untimed batched construction first, so that every kernel either
    # path launches is loaded before the timed runs
    for f in B.construct_batched(*args, oversample=2, device=dev, stream=stream):
        f.close()
    seq_con, seq_samples, facs = timed_construct(
        lambda: [B.construct(w["phase"], X, O, w["tol"], w["leaf"], oversample=2, device=dev, stream=stream)
                 for w, X, O in zip(work, Xs, Os)], keep=True)
    for f, x in zip(facs, xs):
        f.reserve(1 if x.dim() == 1 else x.shape[1], B.C64)
    seq_app = timed_apply(lambda: [f.apply(x, y, stream=stream) for f, x, y in zip(facs, xs, ys)])
    ref = [y.clone() for y in ys[:4]]
    ranks = [f.info()["rank_max"] for f in facs]
    for f in facs:
        f.close()
    del facs
    bat_con, bat_samples, facs = timed_construct(
        lambda: B.construct_batched(*args, oversample=2, device=dev, stream=stream), keep=True)
    for f, x in zip(facs, xs):
        f.reserve(1 if x.dim() == 1 else x.shape[1], B.C64)
    bat_app = timed_apply(lambda: B.apply_batched(facs, xs, ys, stream=stream))
    same = all(torch.equal(a, b) for a, b in zip(ref, ys[:4]))
    graph_app = None
    if stream.cuda_stream:  # capture needs a created stream
        plan = B.ApplyPlan(facs, xs, ys, dtype=B.C64, stream=stream)
        graph_app = timed_apply(lambda: plan.launch(stream))
        same = same and all(torch.equal(a, b) for a, b in zip(ref, ys[:4]))
        plan.close()
    for f in facs:
        f.close()
    return {"instances": len(work), "points": int(sum(w["N"] for w in work)),
            "rank_max_range": [int(min(ranks)), int(max(ranks))],
            "construct_ms_one_by_one": seq_con, "construct_ms_batched": bat_con,
            "construct_ms_samples": {"one_by_one": seq_samples, "batched": bat_samples},
            "apply_ms_one_by_one": seq_app, "apply_ms_batched": bat_app, "apply_ms_graph": graph_app,
            "construct_speedup": seq_con / bat_con, "apply_speedup": seq_app / bat_app,
            "outputs_identical": bool(same)}


def _ablation(B, torch, dev, stream) -> dict:
    """The paper's own ablations on the FIO kernel at N = 2^16 (leaf 16): the
    sampler (Mock-Chebyshev vs uniformly random, t = 1 and 2, tol 1e-6) and
    the fixed truncation rank (tol, k) in {(1e-15, 30), (1e-6, 30)}; epsilon^a
    on 256 exact rows, construction wall time and stored entries.  Measured once."""
    N, leaf = 1 << 16, 16
    ph = I.fio_phase(1.0, 1.0)
    Xh, Oh = I.uniform_grid(N)
    X, O = torch.as_tensor(Xh, device=dev), torch.as_tensor(Oh, device=dev)
    g = torch.as_tensor(I.gaussian_vectors(N, None, 3), device=dev)
    rows = torch.as_tensor(np.sort(np.random.default_rng(2).choice(N, 256, replace=False)), dtype=torch.int32,
                           device=dev)
    ex = B.sample(ph, X, O, rows, torch.arange(N, dtype=torch.int32, device=dev), device=dev) @ g
    variants = {
        "mockcheb_t1": dict(tol=1e-6, oversample=1), "mockcheb_t2": dict(tol=1e-6, oversample=2),
        "random_t1": dict(tol=1e-6, oversample=1, sampler=B.SAMPLER_RANDOM, seed=1),
        "random_t2": dict(tol=1e-6, oversample=2, sampler=B.SAMPLER_RANDOM, seed=1),
        "fixed_k30_tol1e-15": dict(tol=1e-15, kmax=30, oversample=1),
        "fixed_k30_tol1e-6": dict(tol=1e-6, kmax=30, oversample=1),
    }
    out = {}
    for name, kw in variants.items():
        tol = kw.pop("tol")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac = B.construct(ph, X, O, tol, leaf, device=dev, stream=stream, **kw)
        ms = (time.perf_counter() - t0) * 1e3
        y = fac.apply(g)
        info = fac.info()
        out[name] = {"eps_a": float(torch.linalg.norm(y[rows.long()] - ex) / torch.linalg.norm(ex)),
                     "construct_ms": ms, "nnz": int(info["nnz_T"] + info["nnz_S"]), "rank_max": info["rank_max"]}
        fac.close()
    return out


def _example(B, torch, dev, stream, kind: str) -> dict:
    """Examples 3 and 2 of the paper at the workload's size and settings
    (N = 2^20, leaf 16, tol 1e-6, t = 2): the non-uniform Fourier transform
    (rows at random frequencies in [-N/2, N/2), columns at random points in
    [0, 1)) or the Schloemilch kernel J_0(g w) (g_k = (k-1)/N, w_n = n pi).
    Construction wall time and its ID-kernel time, the complex64 1-RHS apply
    (stored bytes / time, as the main line), and epsilon^a on 256 exact rows.
    Measured once."""
    N = WORKLOAD["N"]
    if kind == "nufft":
        ph = I.dft_phase()
        Wh, Xh = I.nufft_points(N, seed=1)
    else:
        ph = I.j0_kernel()
        Wh, Xh = I.schlomilch_points(N)
    Wd, Xd = torch.as_tensor(Wh, device=dev), torch.as_tensor(Xh, device=dev)
    g = torch.as_tensor(I.gaussian_vectors(N, None, 7), device=dev)
    g64 = g.to(torch.complex64)
    y64 = torch.empty_like(g64)
    res = {}
    for it in range(2):  # the first construction warms up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac = B.construct(ph, Wd, Xd, WORKLOAD["tol"], WORKLOAD["leaf"], oversample=WORKLOAD["oversample"],
                          profile=True, device=dev, stream=stream)
        res["construct_ms"] = (time.perf_counter() - t0) * 1e3
        res["id_qr_ms"] = fac.profile(reset=True).get("id_qr", {}).get("ms", 0.0)
        if it == 0:
            fac.close()
    info = fac.info()
    fac.apply(g64, y64, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fac.apply(g64, y64, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    bytes1 = (info["nnz_T"] + info["nnz_S"]) * 8 + 8 * info["n_ids"] + 2 * N * 8
    y = fac.apply(g)
    rows = torch.as_tensor(np.sort(np.random.default_rng(3).choice(N, 256, replace=False)), dtype=torch.int32,
                           device=dev)
    cols = torch.arange(N, dtype=torch.int32, device=dev)
    ex = torch.zeros(256, dtype=torch.complex128, device=dev)
    for c0 in range(0, N, 1 << 16):
        ex += B.sample(ph, Wd, Xd, rows, cols[c0:c0 + (1 << 16)], device=dev) @ g[c0:c0 + (1 << 16)]
    eps_a = float(torch.linalg.norm(y[rows.long()] - ex) / torch.linalg.norm(ex))
    fac.close()
    return {"N": N, "construct_ms": res["construct_ms"], "id_qr_ms": res["id_qr_ms"], "apply1_ms": ms,
            "apply1_gbs": bytes1 / ms / 1e6, "eps_a_256rows": eps_a, "nnz": info["nnz_T"] + info["nnz_S"],
            "rank_min": info["rank_min"], "rank_max": info["rank_max"]}


def _learned(B, torch, dev, stream, n_train: int = 16, n_test: int = 6, keep: int = 8,
             progress: bool = False) -> dict:
    """The learned proposals on the FIO family c(x) = (2 + a sin 2 pi m x)/8
    at N = 2^18 (leaf 16, tol 1e-6, t = 2): the rank network is trained on
    the GPU on ranks from n_train plain constructions (1 in `keep` of their
    IDs), the skeleton network on their skeleton labels (at most 8M
    candidate rows in all); then plain, rank-proposed and rank + skeleton
    proposed constructions of n_test held-out (a, m) are compared (wall
    time, sampled entries, rejected proposals, error on 128 exact rows).
    The default is a reduced run (16 / 6); `--only learned` runs the full
    2000 / 200.  Measured once."""
    N, leaf, tol = 1 << 18, 16, 1e-6
    Xh, Oh = I.uniform_grid(N)
    X, O = torch.as_tensor(Xh, device=dev), torch.as_tensor(Oh, device=dev)
    gen = torch.Generator(device=dev).manual_seed(8)
    t0 = time.perf_counter()
    feats, targ, sfeats, starg = [], [], [], []
    for i, (a, m) in enumerate(I.family_draws(n_train, seed=21)):
        fac = B.construct(I.fio_phase(a, float(m)), X, O, tol, leaf, oversample=2, device=dev, stream=stream)
        H = fac.info()["H"]
        per_call = max(1, 8_000_000 // (n_train * 2 * H))  # skeleton rows kept per level and side
        for side in (B.SIDE_U, B.SIDE_V):
            for t in range(1, H + 1):
                F, tg = B.rank_samples(fac, side, t, device=dev)
                sel = torch.randperm(F.shape[0], generator=gen, device=dev)[: F.shape[0] // keep]
                feats.append(F[sel])
                targ.append(tg[sel])
                F, tg = B.skeleton_samples(fac, side, t, device=dev)
                sel = torch.randperm(F.shape[0], generator=gen, device=dev)[:per_call]
                sfeats.append(F[sel])
                starg.append(tg[sel])
        fac.close()
        if progress and (i + 1) % 100 == 0:
            print(f"learned: {i + 1} training constructions", file=sys.stderr, flush=True)
    F, tg = torch.cat(feats), torch.cat(targ)
    SF, st = torch.cat(sfeats), torch.cat(starg)
    del feats, targ, sfeats, starg
    label_s = time.perf_counter() - t0
    # one call per epoch (Adam's state lives in the network), with a progress
    # line each; the full-scale set is 100x larger, so larger batches and
    # fewer passes
    full = n_train >= 1000
    r_epochs, r_batch = (6, 2048) if full else (20, 512)

    def fit(model, Fm, tm, epochs, batch, seed, name):
        out = []
        for e in range(epochs):
            out.append(float(model.train(Fm, tm, epochs=1, batch=batch, lr=2e-3, seed=seed + 7919 * e,
                                         stream=stream)[0]))
            if progress:
                print(f"learned: {name} epoch {e + 1}/{epochs} loss {out[-1]:.4g}", file=sys.stderr, flush=True)
        return out

    net = B.RankProposer(128, seed=5)
    t0 = time.perf_counter()
    losses = fit(net, F, tg, r_epochs, r_batch, 6, "rank")
    train_s = time.perf_counter() - t0
    snet = B.RankProposer(128, seed=7)
    t0 = time.perf_counter()
    slosses = fit(snet, SF, st, 10, 2048, 8, "skeleton")
    strain_s = time.perf_counter() - t0
    rows = torch.as_tensor(np.sort(np.random.default_rng(1).choice(N, 128, replace=False)), dtype=torch.int32,
                           device=dev)
    cols = torch.arange(N, dtype=torch.int32, device=dev)
    g = torch.as_tensor(I.gaussian_vectors(N, None, 9), device=dev)
    kinds = ("plain", "proposed", "skeleton")
    res = {k: {"ms": [], "sampled": 0, "proposed": 0, "rejected": 0, "err": []} for k in kinds}
    for i, (a, m) in enumerate(I.family_draws(n_test, seed=22)):
        if progress and i % 20 == 0:
            print(f"learned: held-out member {i}", file=sys.stderr, flush=True)
        ph = I.fio_phase(a, float(m))
        ex = torch.zeros(128, dtype=torch.complex128, device=dev)
        for c0 in range(0, N, 1 << 16):
            ex += B.sample(ph, X, O, rows, cols[c0:c0 + (1 << 16)], device=dev) @ g[c0:c0 + (1 << 16)]
        for kind in kinds:
            kw = {}
            if kind != "plain":
                kw = dict(proposer=net, proposal_margin=6, seed=3)
            if kind == "skeleton":
                kw["skeleton_proposer"] = snet
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fac = B.construct(ph, X, O, tol, leaf, oversample=2, device=dev, stream=stream, **kw)
            r = res[kind]
            r["ms"].append((time.perf_counter() - t0) * 1e3)
            info = fac.info()
            r["sampled"] += info["sampled_entries"]
            r["proposed"] += info.get("proposed", 0)
            r["rejected"] += info.get("rejected", 0)
            y = fac.apply(g)
            r["err"].append(float(torch.linalg.norm(y[rows.long()] - ex) / torch.linalg.norm(ex)))
            fac.close()
    net.close()
    snet.close()
    out = {"N": N, "scale": "full (2000 / 200)" if n_train >= 2000 else "reduced",
           "train_constructions": n_train, "train_samples": int(F.shape[0]), "skeleton_train_samples": int(SF.shape[0]),
           "labels_s": label_s, "train_s": train_s, "train_epochs_batch": [r_epochs, r_batch],
           "skeleton_train_s": strain_s,
           "loss_first_last": [float(losses[0]), float(losses[-1])],
           "skeleton_loss_first_last": [float(slosses[0]), float(slosses[-1])], "heldout": n_test}
    base = res["plain"]
    for kind in kinds:
        r = res[kind]
        out[kind] = {"construct_ms": float(np.mean(r["ms"])), "construct_ms_median": float(np.median(r["ms"])),
                     "construct_ms_samples": [round(v, 2) for v in r["ms"][:10]],
                     "err_rows_max": max(r["err"]), "err_rows_median": float(np.median(r["err"]))}
        if kind != "plain":
            out[kind].update({"speedup": float(np.mean(base["ms"]) / np.mean(r["ms"])),
                              "speedup_median": float(np.median(base["ms"]) / np.median(r["ms"])),
                              "sampled_entries_ratio": r["sampled"] / max(base["sampled"], 1),
                              "rejected_frac": r["rejected"] / max(r["proposed"], 1)})
    return out


def _config2(B, torch, dev, stream) -> dict:
    """The N = 2^16 FIO configuration (leaf 16, tol 1e-6, t = 2; FP64
    construction, complex64 applies to 1 and 256 right-hand sides): the
    median of three constructions after a warm-up, event-timed applies in
    every precision, relative errors against the complex128 apply of the same
    factors on 8 probes, and epsilon^a on 256 exact rows.  Measured once."""
    N, leaf, tol, t_os = 1 << 16, 16, 1e-6, 2
    ph = I.fio_phase(1.0, 1.0)
    Xh, Oh = I.uniform_grid(N)
    X, O = torch.as_tensor(Xh, device=dev), torch.as_tensor(Oh, device=dev)
    times, fac = [], None
    for it in range(4):
        if fac is not None:
            fac.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac = B.construct(ph, X, O, tol, leaf, oversample=t_os, device=dev, stream=stream)
        times.append((time.perf_counter() - t0) * 1e3)
    info = fac.info()
    nnz = info["nnz_T"] + info["nnz_S"]
    gen = torch.Generator(device=dev).manual_seed(12)
    out = {"N": N, "construct_ms": float(np.median(times[1:])), "construct_ms_samples": [round(v, 2) for v in times[1:]],
           "nnz": nnz, "rank_min": info["rank_min"], "rank_max": info["rank_max"]}
    fac.reserve(256, B.C128)
    for nrhs in (1, 256):
        xd = (torch.randn(N, nrhs, dtype=torch.complex128, device=dev, generator=gen) * np.sqrt(2.0)).squeeze(1)
        xd = xd.contiguous()
        for name, x, dt in (("c128", xd, B.C128), ("c64", xd.to(torch.complex64), B.C64),
                            ("bf16x3", xd.to(torch.complex64), B.C64_BF16X3)):
            if nrhs == 1 and name == "bf16x3":
                continue
            y = torch.empty_like(x)
            ms = _event_ms(torch, stream, lambda: fac.apply(x, y, dtype=dt, stream=stream))
            rec = {"ms": ms}
            if nrhs == 1:
                rec["gbs"] = (nnz * (16 if name == "c128" else 8) + 8 * info["n_ids"] + 2 * N * x.element_size()) / ms / 1e6
            else:
                rec["gflops"] = 8.0 * nnz * nrhs / ms / 1e6
            out[f"{name}_nrhs{nrhs}"] = rec
        for name in ("c64", "bf16x3"):
            key = f"{name}_nrhs{nrhs}"
            if key in out:
                out[key]["speedup_vs_c128"] = out[f"c128_nrhs{nrhs}"]["ms"] / out[key]["ms"]
    probes = torch.as_tensor(I.gaussian_vectors(N, 8, 5), device=dev)
    y128 = fac.apply(probes)
    p64 = probes.to(torch.complex64)
    for name, dt in (("c64", B.C64), ("bf16x3", B.C64_BF16X3)):
        y = fac.apply(p64, dtype=dt).to(torch.complex128)
        out[f"rel_err_{name}_vs_c128"] = float(torch.linalg.norm(y - y128) / torch.linalg.norm(y128))
    y1 = fac.apply(probes[:, 0].contiguous().to(torch.complex64)).to(torch.complex128)
    out["rel_err_c64_1rhs_vs_c128"] = float(torch.linalg.norm(y1 - y128[:, 0]) / torch.linalg.norm(y128[:, 0]))
    rows = torch.as_tensor(np.sort(np.random.default_rng(0).choice(N, 256, replace=False)), dtype=torch.int32,
                           device=dev)
    ex = B.sample(ph, X, O, rows, torch.arange(N, dtype=torch.int32, device=dev), device=dev) @ probes[:, 0]
    out["eps_a_256rows"] = float(torch.linalg.norm(y128[rows.long(), 0] - ex) / torch.linalg.norm(ex))
    fac.close()
    return out


def _event_ms(torch, stream, fn, warm: bool = True) -> float:
    """Device time of fn() on `stream` between two HIP events (after one untimed run)."""
    if warm:
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


# per-launch HBM traffic of the step's kernels (FETCH_SIZE / WRITE_SIZE passes
# over `bench.py --only step`), keyed "traffic_bytes_per_launch.<record>="
STEP_COUNTERS = os.path.join(ROOT, "profiles", "step_fio_n2p20_counters.md")
STEP_SOURCES = [os.path.join(ROOT, "paper_1809_10573_amd", "csrc", f)
                for f in ("apply.hip", "apply_mfma.hip", "id_batch.hip", "common.hpp", "kernels.hpp")]

def _counted_traffic(path: str, sources: list, key: str) -> float | None:
    """`key` from a committed counter summary, or None when the listed
    sources changed since the counters were taken."""
    import hashlib
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in sources:
        with open(f, "rb") as fh:
            h.update(fh.read())
    kv = dict(l.split("=", 1) for l in lines if l.startswith((key + "=", "source_sha256=")))
    if kv.get("source_sha256", "").strip() != h.hexdigest() or key not in kv:
        return None
    return float(kv[key])


def _only(what: str) -> int:
    """Single pieces of the step for counter runs: the workload's construction
    (twice), its complex64 1-RHS apply (three times, after one construction),
    its 1024-RHS applies (FP32 and BF16 split, once each), one whole step
    (the construction and every apply of the step once, in the step's order,
    with the library's per-launch event times printed for comparison with a
    trace of the same run), or a plain 1 GiB device copy (three times) for
    calibration; or the learned proposal at full scale (2000 training
    constructions, 200 held out)."""
    import torch
    from paper_1809_10573_amd import binding as B
    dev = torch.device("cuda:0")
    if what == "learned":
        res = _learned(B, torch, dev, torch.cuda.current_stream(), n_train=2000, n_test=200, keep=64,
                       progress=True)
        print(json.dumps({"learned": res}), flush=True)
        return 0
    if what == "copy":
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print("copy: 3 x 1 GiB", flush=True)
        return 0
    W = WORKLOAD
    ph = I.fio_phase(W["a"], W["freq"], W["c0"], W["cdiv"])
    Xh, Oh = I.uniform_grid(W["N"])
    X, O = torch.as_tensor(Xh, device=dev), torch.as_tensor(Oh, device=dev)
    if what == "applyn":
        fac = B.construct(ph, X, O, W["tol"], W["leaf"], oversample=W["oversample"], device=dev)
        gen = torch.Generator(device=dev).manual_seed(4)
        XM = torch.randn(W["N"], 1024, dtype=torch.complex64, device=dev, generator=gen)
        YM = torch.empty_like(XM)
        fac.reserve(1024, B.C64)
        fac.apply(XM, YM)
        fac.apply(XM, YM, dtype=B.C64_BF16X3)
        torch.cuda.synchronize()
        print("applyn: one FP32 and one BF16-split apply, 1024 right-hand sides", flush=True)
        fac.close()
        return 0
    if what == "step":
        fac = B.construct(ph, X, O, W["tol"], W["leaf"], oversample=W["oversample"], device=dev, profile=True)
        fac.reserve(1024, B.C128)
        gen = torch.Generator(device=dev).manual_seed(4)
        dt = {"c64": B.C64, "bf16x3": B.C64_BF16X3, "c128": B.C128}
        for name, prec, nrhs in APPLY_KINDS:
            x = torch.randn(W["N"], nrhs, dtype=torch.complex64 if prec != "c128" else torch.complex128,
                            device=dev, generator=gen).squeeze(1).contiguous()
            y = torch.empty_like(x)
            fac.apply(x, y, dtype=dt[prec])
            torch.cuda.synchronize()
            del x, y
            print(f"step: {name} done", file=sys.stderr, flush=True)
        prof = fac.profile(reset=True)
        print(json.dumps({"kernels": {k: {"launches": v["launches"], "ms_per_launch": v["ms"] / v["launches"],
                                          "bytes": v["bytes"], "flops": v["flops"]}
                                      for k, v in sorted(prof.items()) if v["launches"]}}), flush=True)
        fac.close()
        return 0
    if what == "apply1":
        fac = B.construct(ph, X, O, W["tol"], W["leaf"], oversample=W["oversample"], device=dev)
        x = torch.as_tensor(I.gaussian_vectors(W["N"], None, 4), device=dev).to(torch.complex64)
        y = torch.empty_like(x)
        for _ in range(3):
            fac.apply(x, y)
        torch.cuda.synchronize()
        info = fac.info()
        print(f"apply1: 3 applies, nnz {info['nnz_T'] + info['nnz_S']}, n_ids {info['n_ids']}", flush=True)
        fac.close()
        return 0
    for i in range(2):
        fac = B.construct(ph, X, O, W["tol"], W["leaf"], oversample=W["oversample"], device=dev)
        torch.cuda.synchronize()
        print(f"construct {i}: id_flops {fac.info()['id_flops']:.6g}", flush=True)
        fac.close()
    return 0


APPLY_KINDS = [  # (name, dtype, nrhs): every apply of a step, in launch order
    ("c64_nrhs1", "c64", 1), ("c128_nrhs1", "c128", 1),
    ("c64_nrhs256", "c64", 256), ("bf16x3_nrhs256", "bf16x3", 256), ("c128_nrhs256", "c128", 256),
    ("c64_nrhs1024", "c64", 1024), ("bf16x3_nrhs1024", "bf16x3", 1024), ("c128_nrhs1024", "c128", 1024),
]


def _rank_hist(st: dict) -> dict:
    """Per level and side, {rank: IDs} of the nonzero histogram entries."""
    out = {}
    for t, row in enumerate(st["per_level"], start=1):
        for side in ("U", "V"):
            h = row[side]["rank_hist"]
            out[f"{side}{t}"] = {int(r): int(h[r]) for r in np.nonzero(h)[0]}
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the many-instance measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal measurement")
    ap.add_argument("--no-ablation", action="store_true", help="skip the sampler / fixed-rank ablation")
    ap.add_argument("--no-examples", action="store_true",
                    help="skip the non-uniform Fourier transform and Schloemilch lines")
    ap.add_argument("--no-config2", action="store_true", help="skip the N = 2^16 configuration")
    ap.add_argument("--only", choices=["construct", "apply1", "applyn", "step", "copy", "learned"],
                    help="run one piece (counter passes; the full-scale learned proposal)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only; sharding the factorization over several GPUs "
              "is not implemented", file=sys.stderr)
        return 2
    # the oracle's baseline runs first, before anything initializes the GPU
    cpu = None if (args.only or args.no_cpu_baseline) else _cpu_baseline()
    # A step builds a new handle; the library keeps the device memory of a
    # destroyed handle for the next one up to IDBF_CACHE_BYTES.  The step's
    # largest buffers (factors, and the 1024-RHS complex128 apply workspace of
    # about 56 GB) then stay allocated between steps instead of going through
    # hipFree / hipMalloc each time.
    os.environ.setdefault("IDBF_CACHE_BYTES", str(200 << 30))
    if args.only:
        return _only(args.only)

    import torch
    from paper_1809_10573_amd import binding as B

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    W = WORKLOAD
    N = W["N"]
    ph = I.fio_phase(W["a"], W["freq"], W["c0"], W["cdiv"])
    Xh, Oh = I.uniform_grid(N)
    X = torch.as_tensor(Xh, device=dev)
    O = torch.as_tensor(Oh, device=dev)
    stream = torch.cuda.current_stream()
    gen = torch.Generator(device=dev).manual_seed(4)
    # right-hand sides: N(0,1) + i N(0,1) entries (complex randn has variance 1/2 per component)
    xin, yout = {}, {}
    x1d = torch.as_tensor(I.gaussian_vectors(N, None, 4), device=dev)
    xin[("c128", 1)] = x1d
    xin[("c64", 1)] = x1d.to(torch.complex64)
    for nrhs in (256, 1024):
        xd = torch.randn(N, nrhs, dtype=torch.complex128, device=dev, generator=gen) * np.sqrt(2.0)
        xin[("c128", nrhs)] = xd
        xin[("c64", nrhs)] = xd.to(torch.complex64)
    for k, v in xin.items():
        yout[k] = torch.empty_like(v)
    dtypes = {"c64": B.C64, "bf16x3": B.C64_BF16X3, "c128": B.C128}

    tuned: dict = {}  # (name) -> the autotuner's apply configuration, set before each apply

    def step(record):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac = B.construct(ph, X, O, W["tol"], W["leaf"], oversample=W["oversample"], profile=True,
                          device=dev, stream=stream)
        t_con = (time.perf_counter() - t0) * 1e3
        fac.reserve(1024, B.C128)  # the largest apply workspace, before the timed applies
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * len(APPLY_KINDS))]
        for i, (name, prec, nrhs) in enumerate(APPLY_KINDS):
            key = ("c128" if prec == "c128" else "c64", nrhs)
            if name in tuned:  # a host-side setting of the handle, no device work
                fac.set_apply_config(fuse=tuned[name]["fuse"], rhs_iter=tuned[name]["rhs_iter"])
            # the 1-RHS applies run without the library's per-stage event
            # markers (a few microseconds each, 2H + 2 per apply); their
            # per-kernel times come from a profiled apply after the steps
            # (roofline_apply1). Host-side switches, no device work.
            fac.set_profile(nrhs > 1)
            ev[2 * i].record(stream)
            fac.apply(xin[key], yout[key], dtype=dtypes[prec], stream=stream)
            ev[2 * i + 1].record(stream)
            fac.set_profile(True)
        torch.cuda.synchronize()
        if record is not None:
            r = dict(construct_ms=t_con, prof=fac.profile(reset=True), info=fac.info())
            for i, (name, _, _) in enumerate(APPLY_KINDS):
                r[name] = ev[2 * i].elapsed_time(ev[2 * i + 1])
            record.append(r)
        return fac

    for _ in range(args.warmup):
        step(None).close()
    # the apply autotuner on the warm-up factors (outside the timed steps):
    # every many-RHS apply of the step gets its fastest configuration, and the
    # tuner's cache file records it (a fresh file per run)
    tune_file = os.path.join(tempfile.mkdtemp(prefix="idbf_tune_"), "apply_tune.txt")
    # the QR-shape tuner first (it sets the process-wide shapes the timed
    # constructions use), then the apply tuner on factors built with them
    t0 = time.perf_counter()
    tuned_qr = B.tune_construct(ph, X, O, W["tol"], W["leaf"], oversample=W["oversample"],
                                cache_path=tune_file, device=dev, stream=stream)
    tuned_qr["tuning_s"] = time.perf_counter() - t0
    tfac = step(None)
    t0 = time.perf_counter()
    for name, prec, nrhs in APPLY_KINDS:
        if nrhs > 1:
            tuned[name] = tfac.tune_apply(nrhs, dtypes[prec], tune_file, stream=stream)
    tune_s = time.perf_counter() - t0
    tfac.close()
    recs: list = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fac = None
    for _ in range(args.steps):
        if fac is not None:
            fac.close()
        fac = step(recs)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / args.steps

    info = recs[-1]["info"]
    nnz = info["nnz_T"] + info["nnz_S"]
    construct_ms = float(np.mean([r["construct_ms"] for r in recs]))
    apply = {}
    for name, prec, nrhs in APPLY_KINDS:
        ms = float(np.mean([r[name] for r in recs]))
        rec = {"ms": ms}
        if nrhs == 1:
            elem = 16 if prec == "c128" else 8
            rec["gbs"] = (nnz * elem + 8 * info["n_ids"] + 2 * N * elem) / ms / 1e6
            rec["frac_hbm_peak"] = rec["gbs"] / HBM_PEAK_GBS
        else:
            rec["gflops"] = 8.0 * nnz * nrhs / ms / 1e6
            peak = {"c64": FP32_MFMA_PEAK, "bf16x3": BF16_MFMA_PEAK, "c128": FP64_MFMA_PEAK}[prec]
            rec["frac_peak"] = rec["gflops"] * 1e9 / peak
            rec["peak"] = {"c64": "FP32 MFMA", "bf16x3": "BF16 MFMA", "c128": "FP64 MFMA"}[prec]
            rec["tuned"] = ({"fuse": tuned[name]["fuse"] if prec != "c128" else None,  # no fused complex128 path
                             "rhs_iter": tuned[name]["rhs_iter"]} if name in tuned else None)
        apply[name] = rec
    for name, prec, nrhs in APPLY_KINDS:
        if prec != "c128":
            apply[name]["speedup_vs_c128"] = apply[f"c128_nrhs{nrhs}"]["ms"] / apply[name]["ms"]
    value = apply["c64_nrhs1"]["gbs"]

    # per-kernel aggregates over the timed steps
    agg: dict = {}
    for r in recs:
        for name, st in r["prof"].items():
            a = agg.setdefault(name, dict(launches=0, ms=0.0, bytes=0.0, flops=0.0))
            for k in a:
                a[k] += st[k]
    dom_name = max(agg, key=lambda k: agg[k]["ms"])
    dom = agg[dom_name]
    if dom_name == "id_qr":
        achieved = dom["flops"] / (dom["ms"] * 1e-3) / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=FP64_VALU_PEAK / 1e12, unit="TFLOP/s")
    elif dom_name.startswith("applyn") or dom_name.startswith("applyb"):
        # complex128 many-RHS stages run on FP64 MFMA, complex64 on FP32 MFMA
        achieved = dom["flops"] / (dom["ms"] * 1e-3) / 1e12
        peak = (FP64_MFMA_PEAK if dom_name.startswith("applynd") else
                FP32_MFMA_PEAK if dom_name.startswith("applyn") else BF16_MFMA_PEAK)
        roof = dict(bound="mfma", achieved=achieved, peak=peak / 1e12, unit="TFLOP/s")
    else:
        achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = _counted_traffic(STEP_COUNTERS, STEP_SOURCES, "traffic_bytes_per_launch." + dom_name)
    roof["kernel"] = dom_name
    roof["launches_per_step"] = dom["launches"] / len(recs)

    # accuracy (outside the timed region): every precision against the FP64
    # (complex128) apply of the same factors on 8 probe vectors, and the
    # paper's epsilon^a on 256 rows
    probes = torch.as_tensor(I.gaussian_vectors(N, 8, 5), device=dev)
    p64 = probes.to(torch.complex64).contiguous()
    y128 = fac.apply(probes)
    errs = {}
    for prec in ("c64", "bf16x3"):
        y = fac.apply(p64, dtype=dtypes[prec]).to(torch.complex128)
        errs[prec] = float(torch.linalg.norm(y - y128) / torch.linalg.norm(y128))
    y1 = fac.apply(p64[:, 0].contiguous()).to(torch.complex128)
    errs["c64_1rhs"] = float(torch.linalg.norm(y1 - y128[:, 0]) / torch.linalg.norm(y128[:, 0]))
    for name, prec, nrhs in APPLY_KINDS:
        if prec != "c128":
            apply[name]["rel_err_vs_c128"] = errs["c64_1rhs" if nrhs == 1 else prec]
    rows = np.sort(np.random.default_rng(0).choice(N, 256, replace=False))
    ex = torch.zeros(256, dtype=torch.complex128, device=dev)
    cols = torch.arange(N, dtype=torch.int32, device=dev)
    rows_d = torch.as_tensor(rows, dtype=torch.int32, device=dev)
    for c0 in range(0, N, 1 << 16):
        K = B.sample(ph, X, O, rows_d, cols[c0:c0 + (1 << 16)], device=dev)
        ex += K @ probes[c0:c0 + (1 << 16), 0]
    eps_a = float(torch.linalg.norm(y128[rows, 0] - ex) / torch.linalg.norm(ex))
    st = fac.stats()

    out = {
        "metric": METRIC, "value": value, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 apply (value) / c128 and bf16x3 applies / f64 construct",
        "data": "synthetic",
        "config": {"workload": "FIO exp(2 pi i (x xi + (2+sin 2 pi x)/8 |xi|)), uniform grid",
                   "N": N, "leaf": W["leaf"], "tol": W["tol"], "oversample": W["oversample"],
                   "nrhs": [1, 256, 1024]},
        "construct_ms": construct_ms, "apply": apply, "apply_tuning_s": tune_s,
        "qr_shapes": {"mask": tuned_qr["mask"], "id_qr_ms": tuned_qr["ms"], "tuning_s": tuned_qr["tuning_s"]},
        "apply1_ms": apply["c64_nrhs1"]["ms"], "apply1_c128_ms": apply["c128_nrhs1"]["ms"],
        "applyn_ms": apply["c64_nrhs1024"]["ms"], "applyn_gflops": apply["c64_nrhs1024"]["gflops"],
        "applyb_ms": apply["bf16x3_nrhs1024"]["ms"], "applyb_gflops": apply["bf16x3_nrhs1024"]["gflops"],
        "id_fp64_tflops": agg.get("id_qr", {}).get("flops", 0) / max(agg.get("id_qr", {}).get("ms", 1), 1e-9) / 1e9,
        "rel_err_c64_vs_c128": errs["c64"], "rel_err_bf16x3_vs_c128": errs["bf16x3"], "eps_a_256rows": eps_a,
        "nnz": nnz, "rank_max": info["rank_max"],
        "rank_hist": _rank_hist(st),
        "tall_ids": int(sum(row[s]["tall"] for row in st["per_level"] for s in "UV")),
        "kernels": {k: {"launches_per_step": v["launches"] / len(recs),
                        "ms_per_step": v["ms"] / len(recs)} for k, v in sorted(agg.items())},
        "roofline": roof,
        "roofline_apply1": None,
        "cpu_baseline": cpu,
    }
    # 1-RHS apply roofline: the three stage kernels of one complex64 1-RHS apply
    x1, y1b = xin[("c64", 1)], yout[("c64", 1)]
    fac.apply(x1, y1b)
    torch.cuda.synchronize()
    fac.profile(reset=True)
    fac.apply(x1, y1b)
    p1 = fac.profile(reset=True)
    tb = sum(v["bytes"] for k, v in p1.items() if k.startswith("apply"))
    tm = sum(v["ms"] for k, v in p1.items() if k.startswith("apply"))
    out["roofline_apply1"] = {"bound": "hbm", "achieved": tb / tm / 1e6, "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": tb / tm / 1e6 / HBM_PEAK_GBS,
                              "traffic": _counted_traffic(STEP_COUNTERS, STEP_SOURCES,
                                                          "traffic_bytes_per_apply.c64_nrhs1"),
                              "kernels": {k: v["ms"] for k, v in p1.items()}}
    # the 1-RHS applies issued back to back, eagerly and replayed from a
    # captured HIP graph (a one-instance apply plan): 20 of each between two
    # events; the graph removes the host launch of each of the 2H + 1 stages
    reps = 20
    replay = {}
    cap = torch.cuda.Stream()  # capture needs a stream of its own (default priority)
    fac.set_profile(False)  # no event markers on either side (the graph records none)
    torch.cuda.synchronize()
    for name, key in (("c64_nrhs1", ("c64", 1)), ("c128_nrhs1", ("c128", 1))):
        xk, yk = xin[key], yout[key]
        plan = B.ApplyPlan([fac], [xk], [yk], stream=cap)
        eager_ms = _event_ms(torch, cap, lambda: [fac.apply(xk, yk, stream=cap) for _ in range(reps)]) / reps
        graph_ms = _event_ms(torch, cap, lambda: [plan.launch(cap) for _ in range(reps)]) / reps
        plan.close()
        elem = 16 if key[0] == "c128" else 8
        gb = (nnz * elem + 8 * info["n_ids"] + 2 * N * elem) / 1e9
        replay[name] = {"eager_ms": eager_ms, "graph_ms": graph_ms, "graph_gbs": gb / graph_ms * 1e3,
                        "graph_frac_hbm_peak": gb / graph_ms * 1e3 / HBM_PEAK_GBS}
    out["apply1_replay"] = replay
    # adjoint apply y = K~^H x on the same factors (measured once), with the
    # adjoint identity as a check
    adj = {}
    for name, prec, nrhs in APPLY_KINDS:
        if nrhs == 256:
            continue
        key = ("c128" if prec == "c128" else "c64", nrhs)
        adj[name] = _event_ms(torch, stream, lambda: fac.apply_adjoint(xin[key], yout[key], dtype=dtypes[prec],
                                                                       stream=stream))
    p0 = probes[:, 0].contiguous()
    pb = probes[:, 1].contiguous()
    ident = abs(complex(torch.vdot(pb, fac.apply(p0)) - torch.vdot(fac.apply_adjoint(pb), p0)))
    ident /= float(torch.linalg.norm(pb) * torch.linalg.norm(fac.apply(p0)))
    out["adjoint"] = {"ms": adj, "identity_rel_err_c128": ident}
    fac.close()
    del xin, yout
    torch.cuda.empty_cache()
    if not args.no_config2:
        out["config2"] = _config2(B, torch, dev, stream)
    if not args.no_batched:
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            out["batched"] = _batched(B, torch, dev, side)
    if not args.no_learned:
        out["learned"] = _learned(B, torch, dev, stream)
    if not args.no_ablation:
        out["ablation"] = _ablation(B, torch, dev, stream)
    if not args.no_examples:
        out["nufft"] = _example(B, torch, dev, stream, "nufft")
        out["schlomilch_j0"] = _example(B, torch, dev, stream, "j0")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
