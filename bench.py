"""Benchmark: QP time-to-solution, PCG iterations/s and SpMV HBM GB/s vs peak.

One step = one whole QP solve (qp_solve: start point, residuals, every PCG
direction, recovery, ratio test, update, barrier rule) of the banded-dose QP
with n = 20,000 spots, J 400,000 x 20,000 (40M nnz), A 2,000 x 20,000 at 2%,
bounds [0, 50], PCG tolerance 1e-8, with the library's default settings
(captured PCG graphs).  Problem data are resident in HBM (created once by
qp_create) before the timed region.  One more solve on a second handle with
per-kernel HIP events gives the SpMV kernel durations of the roofline; a
child process measures the streaming-read ceiling with torch.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64]
                    [--scale 1.0] [--no-cpu-baseline]

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QP time-to-solution & PCG iters/s; SpMV HBM GB/s vs peak, mixed vs FP64"
HBM_PEAK_GBS = 8000.0


def spmv_bytes(n, nJ, m, nnzJ, nnzA, vbytes=8, fmt=0):
    """Algorithmic HBM bytes of one operator product, per kernel.

    Each matrix value and index read once, row pointers once, every dense
    vector read or written once (gathered vectors counted once).  fmt = 0: CSR
    (int32 column index per nonzero), a J pass and a J^T pass that each read
    the values.  fmt = 1: line format in a PCG product, a line pass that reads
    the values once (one int32 column id per 64-row line slot), gathers z and
    p, and writes one double per slot, and forms u from A z and A p (five
    m-vectors: A z, A p read and written, Sigma_A, u); then a spot pass that
    reads one int32 slot id and that double per slot, A^T, u, z, p and
    Sigma_x, and writes p and q."""
    if fmt == 1:
        slots = nnzJ // 64
        lines = nJ // 64
        fwd = (nnzJ * vbytes + slots * 4 + (lines + 1) * 4 + nJ * 8 + 2 * n * 8 + slots * 8
               + 5 * m * 8)
        bwd = (n + 1) * 4 + slots * 4 + slots * 8 + nnzA * 12 + (n + 1) * 4 + m * 8 + n * 8 * 5
        return fwd, bwd
    jf = nnzJ * (vbytes + 4) + (nJ + 1) * 4
    jb = nnzJ * (vbytes + 4) + (n + 1) * 4
    fwd = jf + n * 8 + nJ * 8 + nJ * 8 + nnzA * 12 + (m + 1) * 4 + m * 8 + m * 8
    bwd = jb + nJ * 8 + nnzA * 12 + (n + 1) * 4 + m * 8 + n * 8 * 3
    return fwd, bwd


def cpu_baseline(prob, ipm_iters):
    """The FP64 dense-Cholesky oracle on a bounded sample of the same QP: the
    dense Hessian formation plus one IPM iteration (condensed matrix,
    Cholesky, recovery, update), extrapolated to a whole solve of `ipm_iters`
    iterations."""
    import threadpoolctl
    import oracle
    from oracle import ipm_dense as O

    cores = len(os.sched_getaffinity(0))
    with threadpoolctl.threadpool_limits(cores):
        t0 = time.perf_counter()
        H = oracle.hessian_dense(prob)
        t1 = time.perf_counter()
        zeta = O.objective_scale(prob, H)
        H /= zeta
        import copy
        sp_ = copy.copy(prob)
        sp_.p = prob.p / zeta
        G = O.make_groups(sp_)
        x, s, lam = O.initial_point(sp_, G)
        mu = float(sum(s[g] @ lam[g] for g in O.GROUPS) / G.m_tot())
        t2 = time.perf_counter()
        Hx, rH, rg, rc = O.residuals(sp_, G, H, x, s, lam, mu)
        dx, ds, dl = O.newton_direction(sp_, G, H, x, s, lam, mu, Hx, rg)
        ax = O.max_step(s, ds, 0.995)
        x = x + ax * dx
        t3 = time.perf_counter()
        used = threadpoolctl.threadpool_info()
    nthreads = max([u.get("num_threads", 1) for u in used] + [1])
    t_qp = (t1 - t0) + (t2 - t1) + ipm_iters * (t3 - t2)
    return {"value": 1.0 / t_qp, "unit": "QP/s", "cores": int(nthreads), "kind": "oracle",
            "sample": (f"dense H formation ({t1 - t0:.1f} s) + 1 IPM iteration ({t3 - t2:.1f} s) of the "
                       f"FP64 dense-Cholesky oracle on the same n={prob.n} QP, extrapolated to "
                       f"{ipm_iters} IPM iterations"),
            "seconds_per_qp_extrapolated": t_qp}


def kernel_source_hash():
    """Hash of the operator kernels' code (comments and blank lines left out,
    so that a comment edit does not void the committed counter summary)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("device_common.hpp", "ipm_kernels.hpp", "line_kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2405_03584_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def counter_traffic(kernel_tag, precision):
    """HBM bytes per launch from the committed counter summary, or None when
    the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"op_traffic_config2_{precision}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    for name, v in rec["kernels"].items():
        if name.split("<")[0] == kernel_tag:
            return v["hbm_bytes"]
    return None


def operator_only(args, prob):
    """Repeated operator products q = K v at a fixed seeded Sigma (one forward
    and one backward SpMV launch each)."""
    from paper_2405_03584_amd import qpgpu
    import qpsynth
    it = qpsynth.random_iterate(prob, 1)
    h = qpgpu.qp_create_from_problem(prob, settings=qpgpu.qp_default_settings(timing=1))
    y, info = qpgpu.qp_operator_apply(h, it["sigma_x"], it["sigma_A"], it["v"], precision=args.precision,
                                      reps=args.reps)
    n, m, nJ = prob.n, prob.m, prob.J.shape[0]
    vbytes = {"fp64": 8, "fp32": 4, "bf16": 2}[args.precision]
    fmt = info["spmv_format"]
    bf, bb = spmv_bytes(n, nJ, m, int(prob.J.nnz), int(prob.A.nnz), vbytes, fmt)
    cf, cb = spmv_bytes(n, nJ, m, int(prob.J.nnz), int(prob.A.nnz), vbytes, 0)
    fus = 1e3 * info["t_spmv_fwd_ms"] / max(info["n_spmv_fwd"], 1)
    bus = 1e3 * info["t_spmv_bwd_ms"] / max(info["n_spmv_bwd"], 1)
    print(json.dumps({"mode": "operator", "precision": args.precision, "reps": args.reps,
                      "format": ["csr", "line"][fmt],
                      "fwd_us": fus, "bwd_us": bus, "fwd_GBs": bf / fus / 1e3, "bwd_GBs": bb / bus / 1e3,
                      "fwd_bytes": bf, "bwd_bytes": bb,
                      "csr_equivalent_fwd_GBs": cf / fus / 1e3, "csr_equivalent_bwd_GBs": cb / bus / 1e3,
                      "checksum": float(np.abs(y).sum())}), flush=True)


def batch_bench(args):
    """The uneven batch: `count` members of the 64-QP set, created once, then
    solved together (qp_solve_batch) per step."""
    import qpsynth
    from paper_2405_03584_amd import qpgpu
    t0 = time.perf_counter()
    probs = [qpsynth.config4_instance(i) for i in range(args.count)]
    nnz = sum(int(p.J.nnz) for p in probs)
    print(f"[bench] generated {len(probs)} QPs, n in [{min(p.n for p in probs)}, {max(p.n for p in probs)}], "
          f"{nnz} nnz of J in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    st = qpgpu.qp_default_settings(precision=args.precision)
    hs = [qpgpu.qp_create_from_problem(p, settings=st) for p in probs]
    print(f"[bench] created handles", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        s, xs, infos = qpgpu.qp_solve_batch(hs)
        print(f"[bench] warmup {i}: status={s}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    all_infos = []
    for i in range(args.steps):
        s, xs, infos = qpgpu.qp_solve_batch(hs)
        all_infos += infos
        print(f"[bench] step {i}: status={s} pcg={sum(f['pcg_iters'] for f in infos)}", file=sys.stderr, flush=True)
    el = time.perf_counter() - t0
    ok = all(f["status"] == qpgpu.QP_OK for f in all_infos)
    # the same handles solved one after another (one stream busy at a time)
    t1 = time.perf_counter()
    for h in hs:
        qpgpu.qp_solve(h)
    seq = time.perf_counter() - t1
    print(f"[bench] sequential: {1e3 * seq:.1f} ms", file=sys.stderr, flush=True)
    print(json.dumps({"metric": METRIC, "value": args.count * args.steps / el, "unit": "QP/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": args.precision, "data": "synthetic",
                      "config": {"workload": f"batch of {args.count} uneven banded-dose QPs "
                                             f"(n in [2000, 20000], {nnz} nnz of J in all)",
                                 "precision": args.precision},
                      "status_ok": ok,
                      "sequential_ms": 1e3 * seq,
                      "batch_speedup_vs_sequential": seq / (el / args.steps),
                      "ipm_iters_total": sum(f["ipm_iters"] for f in all_infos),
                      "pcg_iters_total": sum(f["pcg_iters"] for f in all_infos)}), flush=True)


def sqp_bench(args):
    """A sequence of `seq_len` SQP sub-problems on the n = 20,000 banded-dose
    QP (rank-2 growth of the quasi-Newton term per step): one handle, per
    step qp_update_hessian + qp_solve (or qp_solve_from the previous
    minimiser with --warm 1).  For comparison, one sub-problem through
    qp_create + qp_solve, the cost without a resident handle."""
    import qpsynth
    from paper_2405_03584_amd import qpgpu
    base = qpsynth.config2(scale=args.scale)
    seq = qpsynth.sqp_sequence(base, args.seq_len + args.warmup)
    st = qpgpu.qp_default_settings(precision=args.precision)
    h = qpgpu.qp_create_from_problem(seq[0], settings=st)
    x_prev = None

    def step(q, first):
        nonlocal x_prev
        if not first:
            qpgpu.qp_update_hessian(h, q.gamma, q.p, q.U, q.w)
        r = qpgpu.qp_solve_from(h, x_prev) if args.warm else qpgpu.qp_solve(h)
        x_prev = r.x
        return r

    for i in range(args.warmup):
        r = step(seq[i], i == 0)
        print(f"[bench] warmup {i}: status={r.status} ipm={r.info['ipm_iters']}", file=sys.stderr, flush=True)
    infos = []
    t0 = time.perf_counter()
    for i in range(args.warmup, args.warmup + args.seq_len):
        r = step(seq[i], i == 0)
        infos.append(r.info)
        print(f"[bench] sub-problem {i} k={seq[i].k}: status={r.status} ipm={r.info['ipm_iters']} "
              f"pcg={r.info['pcg_iters']}", file=sys.stderr, flush=True)
    el = time.perf_counter() - t0
    t1 = time.perf_counter()
    h2 = qpgpu.qp_create_from_problem(seq[-1], settings=st)
    qpgpu.qp_solve(h2)
    fresh = time.perf_counter() - t1
    h2.close()
    ok = all(f["status"] == qpgpu.QP_OK for f in infos)
    print(json.dumps({"metric": METRIC, "value": args.seq_len / el, "unit": "QP/s", "n_gpus": 1,
                      "steps": args.seq_len, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.seq_len,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": args.precision, "data": "synthetic",
                      "config": {"workload": f"SQP sequence of {args.seq_len} sub-problems on the banded-dose "
                                             f"QP n={base.n} (quasi-Newton rank +2 per step, "
                                             f"{'warm' if args.warm else 'cold'} start)",
                                 "precision": args.precision},
                      "status_ok": ok,
                      "create_plus_solve_ms": 1e3 * fresh,
                      "ipm_iters": [f["ipm_iters"] for f in infos],
                      "pcg_iters": [f["pcg_iters"] for f in infos]}), flush=True)


def stream_ceiling():
    """Measured streaming-read ceiling in GB/s, from `--mode stream` run in a
    child process (torch brings its own HIP runtime, which must not share a
    process with the library's)."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--mode", "stream"], capture_output=True,
                       text=True, timeout=300)
    if r.returncode != 0:
        print(f"[bench] stream ceiling failed: {r.stderr[-400:]}", file=sys.stderr, flush=True)
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])["read_GBs"]


def stream_read(args):
    """A 1 GiB FP64 tensor summed by torch (each byte read once), best of 5
    after a warm-up: the streaming-read ceiling the kernels are compared to."""
    import torch
    x = torch.ones((1 << 30) // 8, dtype=torch.float64, device="cuda")
    x.sum()
    torch.cuda.synchronize()
    best = None
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        x.sum()
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    print(json.dumps({"mode": "stream", "bytes": 1 << 30, "ms": best, "read_GBs": (1 << 30) / (best * 1e-3) / 1e9}),
          flush=True)


def copy_calibration(args):
    """A plain device-to-device copy of a known byte count with torch's copy
    kernel: what the HBM counters read for it calibrates the counter scale."""
    import torch
    nbytes = 480_000_000
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes,
                      "reps": args.reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--log", type=int, default=1, help="per-IPM-iteration progress on stderr")
    ap.add_argument("--mode", default="solve", choices=["solve", "operator", "copy", "stream"],
                    help="solve: whole QP solves (the benchmark); operator: repeated operator "
                         "products only (for counter runs); copy: a plain device copy of the "
                         "J value+index bytes (counter calibration)")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--graphs", type=int, default=1, choices=[0, 1],
                    help="1: PCG iterations replayed as captured HIP graphs (the production setting); "
                         "0: direct launches (for kernel-trace and counter runs)")
    ap.add_argument("--workload", default="config2", choices=["config2", "config5", "batch", "sqp"],
                    help="config2: banded-dose QP n=20,000 (default, the benchmark line); config5: "
                         "n=60,000, BF16-valued J with 200M nnz and a rank-20 term; batch: the 64 "
                         "uneven QPs (n in [2000, 20000]) solved together by qp_solve_batch")
    ap.add_argument("--count", type=int, default=64, help="batch size for --workload batch")
    ap.add_argument("--seq-len", type=int, default=6, help="sub-problems timed for --workload sqp")
    ap.add_argument("--warm", type=int, default=0, choices=[0, 1],
                    help="--workload sqp: start each solve at the previous minimiser")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (single-GPU build)",
              file=sys.stderr)
        sys.exit(2)

    import qpsynth
    from paper_2405_03584_amd import qpgpu

    if args.mode == "copy":
        return copy_calibration(args)
    if args.mode == "stream":
        return stream_read(args)
    if args.workload == "batch":
        return batch_bench(args)
    if args.workload == "sqp":
        return sqp_bench(args)
    ceiling = stream_ceiling() if args.mode == "solve" else None   # before this process touches the GPU
    t0 = time.perf_counter()
    prob = qpsynth.config5(scale=args.scale) if args.workload == "config5" else qpsynth.config2(scale=args.scale)
    if args.mode == "operator":
        return operator_only(args, prob)
    n, m, nJ = prob.n, prob.m, prob.J.shape[0]
    nnzJ, nnzA = int(prob.J.nnz), int(prob.A.nnz)
    print(f"[bench] generated n={n} nJ={nJ} nnzJ={nnzJ} m={m} nnzA={nnzA} in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    # the timed solves use the production settings (captured PCG graphs, no
    # per-kernel events); one extra solve on a second handle with timing = 1
    # gives the SpMV kernel durations for the roofline
    settings = qpgpu.qp_default_settings(precision=args.precision, log_level=args.log, graphs=args.graphs)
    t0 = time.perf_counter()
    h = qpgpu.qp_create_from_problem(prob, settings=settings)
    t_create = time.perf_counter() - t0
    print(f"[bench] qp_create {t_create:.2f}s", file=sys.stderr, flush=True)

    for i in range(args.warmup):
        r = qpgpu.qp_solve(h)
        print(f"[bench] warmup {i}: status={r.status} ipm={r.info['ipm_iters']} "
              f"pcg={r.info['pcg_iters']} {r.info['t_solve_ms']:.1f} ms", file=sys.stderr, flush=True)

    infos = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = qpgpu.qp_solve(h)
        infos.append(r.info)
        print(f"[bench] step {i}: status={r.status} ipm={r.info['ipm_iters']} pcg={r.info['pcg_iters']} "
              f"{r.info['t_solve_ms']:.1f} ms", file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t0
    x_last = r.x
    status_ok = all(i["status"] == qpgpu.QP_OK for i in infos)

    pcg_iters = sum(i["pcg_iters"] for i in infos)
    pcg_ms = sum(i["t_pcg_ms"] for i in infos)
    ht = qpgpu.qp_create_from_problem(prob, settings=qpgpu.qp_default_settings(precision=args.precision,
                                                                              timing=1))
    rt = qpgpu.qp_solve(ht)
    print(f"[bench] timing solve: status={rt.status} pcg={rt.info['pcg_iters']} {rt.info['t_solve_ms']:.1f} ms",
          file=sys.stderr, flush=True)
    tinfo = [rt.info]
    fwd_ms = sum(i["t_spmv_fwd_ms"] for i in tinfo)
    bwd_ms = sum(i["t_spmv_bwd_ms"] for i in tinfo)
    nf = sum(i["n_spmv_fwd"] for i in tinfo)
    nb = sum(i["n_spmv_bwd"] for i in tinfo)
    vbytes = {"fp64": 8, "fp32": 4, "bf16": 2}[args.precision]
    fmt = infos[-1]["spmv_format"]
    bf, bb = spmv_bytes(n, nJ, m, nnzJ, nnzA, vbytes, fmt)
    cf, cb = spmv_bytes(n, nJ, m, nnzJ, nnzA, vbytes, 0)
    fwd_us = 1e3 * fwd_ms / max(nf, 1)
    bwd_us = 1e3 * bwd_ms / max(nb, 1)
    gbs_f = bf / (fwd_us * 1e-6) / 1e9
    gbs_b = bb / (bwd_us * 1e-6) / 1e9
    if fmt == 1:
        names = ("k_line_pass (J p, W scaling and per-slot J^T contributions from one read of J; u from A z and A p)",
                 "k_spot_pass (per-spot J^T sums, A^T u, epilogue and p.q partials)")
    else:
        names = ("k_op_fwd (J + A SpMV, fused W / Sigma_A scaling)",
                 "k_op_bwd (J^T + A^T SpMV, fused epilogue and p.q partials)")
    dom = (names[1], bb, bwd_us, gbs_b) if bwd_us >= fwd_us else (names[0], bf, fwd_us, gbs_f)

    parity = None
    gold = os.path.join(ROOT, "tests", "golden", "config2_oracle.json")
    if args.workload == "config2" and args.scale == 1.0 and os.path.exists(gold):
        g = json.load(open(gold))
        step = g["sample_index_step"]
        xs = np.array(g["x_sample"])
        parity = {"x_sample_max_abs_err_vs_oracle": float(np.abs(x_last[::step] - xs).max()),
                  "objective_rel_err_vs_oracle": abs(infos[-1]["objective"] - g["objective"]) / abs(g["objective"])}

    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "QP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32 values, f32 accum, f64 scalars",
                  "bf16": "bf16 values, f32 accum, f64 scalars"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"banded-dose QP n={n} (J {nJ}x{n}, {nnzJ} nnz; A {m}x{n}, {nnzA} nnz; "
                               f"bounds [0,50]; PCG tol 1e-8"
                               + (f"; rank-{prob.k} term; BF16-valued J" if prob.k else "") + ")",
                   "precision": args.precision, "scale": args.scale},
        "time_to_solution_ms": 1e3 * elapsed / args.steps,
        "ipm_iters": infos[-1]["ipm_iters"],
        "pcg_iters_per_qp": pcg_iters / args.steps,
        "pcg_iters_per_s": pcg_iters / (pcg_ms * 1e-3) if pcg_ms > 0 else None,
        "status_ok": status_ok,
        "spmv": {"format": ["csr", "line"][fmt], "fwd_us": fwd_us, "bwd_us": bwd_us, "fwd_GBs": gbs_f,
                 "bwd_GBs": gbs_b, "fwd_bytes": bf, "bwd_bytes": bb, "timed_launches": nb,
                 "csr_equivalent_fwd_GBs": cf / (fwd_us * 1e-6) / 1e9,
                 "csr_equivalent_bwd_GBs": cb / (bwd_us * 1e-6) / 1e9},
        "roofline": {"bound": "hbm", "kernel": dom[0], "achieved": dom[3], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dom[3] / HBM_PEAK_GBS,
                     "traffic": (counter_traffic(dom[0].split()[0], args.precision)
                                 if args.scale == 1.0 and args.workload == "config2" else None),
                     "bytes_per_launch": dom[1], "avg_launch_us": dom[2],
                     "stream_read_ceiling_GBs": ceiling,
                     "frac_of_stream_ceiling": dom[3] / ceiling if ceiling else None},
        "create_s": t_create,
        "parity": parity,
    }
    # the paper's speedups are over a commercial CPU solver on its own clinical
    # QPs and machines: printed beside ours for context, not compared
    out["paper_context"] = {
        "speedup_over_raystation_qp_solver": {"proton_head_and_neck_200_qps": 4.4,
                                              "vmat_head_and_neck_33_qps": 1.4},
        "paper_hardware": "paper's solver on an RTX 4080 GPU with a Ryzen 9 7900X host; RayStation 2024A "
                          "on an Intel i9-7940X",
        "precision": "FP64"}
    if not args.no_cpu_baseline and args.workload == "config2":
        print("[bench] cpu baseline (oracle sample)...", file=sys.stderr, flush=True)
        iters = infos[-1]["ipm_iters"]
        if args.scale == 1.0 and os.path.exists(gold):
            iters = json.load(open(gold))["ipm_iters"]
        out["cpu_baseline"] = cpu_baseline(prob, iters)
        out["speedup_over_cpu_oracle"] = out["value"] / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
