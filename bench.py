"""Benchmark: QP time-to-solution, PCG iterations/s and SpMV HBM GB/s vs peak,
mixed precision vs FP64.

One step = one whole QP solve (qp_solve: start point, residuals, every PCG
direction, recovery, ratio test, update, barrier rule) of the banded-dose QP
with n = 20,000 spots, J 400,000 x 20,000 (40M nnz), A 2,000 x 20,000 at 2%,
bounds [0, 50], PCG tolerance 1e-8, with the library's default settings
(captured PCG graphs).  Problem data are resident in HBM (created once by
qp_create) before the timed region.  `value` is the FP64 (or --precision)
rate; the same QP is then timed with BF16 and FP32 values of J
(`by_precision`, `mixed_vs_fp64`).  One more solve per precision on a handle
with per-kernel HIP events gives the operator kernels' durations for the
roofline, the general CSR path's operator is timed on the same QP
(`csr_operator`), a child process measures the streaming-read ceiling with
torch, the 64 uneven QPs of the batch workload are solved together by
qp_solve_batch in each precision (`batch64`), and the FP64 dense-Cholesky
oracle solves the same QP on the host cores (`cpu_baseline`).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64]
                    [--scale 1.0] [--cpu-baseline full|sample|none] [--mixed 1] [--csr 1] [--batch 1]

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


def cpu_baseline(prob, mode="full", ipm_iters=None):
    """The FP64 dense-Cholesky oracle on the host cores, on the same QP.
    mode "full": the whole oracle solve (dense H formation, then every IPM
    iteration to convergence), one progress line per iteration on stderr;
    mode "sample": dense H formation plus one IPM iteration, extrapolated to
    `ipm_iters` iterations."""
    import threadpoolctl
    import oracle
    from oracle import ipm_dense as O

    cores = len(os.sched_getaffinity(0))
    with threadpoolctl.threadpool_limits(cores):
        t0 = time.perf_counter()
        H = oracle.hessian_dense(prob)
        t1 = time.perf_counter()
        print(f"[bench] oracle: dense H in {t1 - t0:.1f} s", file=sys.stderr, flush=True)
        if mode == "full":
            def report(it, mu, rn):
                print(f"[bench] oracle IPM iteration {it}: mu {mu:.2e} rnorm {rn:.2e} "
                      f"({time.perf_counter() - t1:.0f} s)", file=sys.stderr, flush=True)
            res = oracle.solve(prob, H=H, progress=report)
            t2 = time.perf_counter()
            used = threadpoolctl.threadpool_info()
            t_qp = t2 - t0
            sample = (f"the whole FP64 dense-Cholesky oracle solve of the same n={prob.n} QP: dense H "
                      f"formation ({t1 - t0:.1f} s) + {res.iters} IPM iterations ({t2 - t1:.1f} s)")
            extra = {"oracle_ipm_iters": int(res.iters), "oracle_converged": bool(res.converged),
                     "oracle_objective": res.objective}
        else:
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
            t_qp = (t1 - t0) + (t2 - t1) + ipm_iters * (t3 - t2)
            sample = (f"dense H formation ({t1 - t0:.1f} s) + 1 IPM iteration ({t3 - t2:.1f} s) of the "
                      f"FP64 dense-Cholesky oracle on the same n={prob.n} QP, extrapolated to "
                      f"{ipm_iters} IPM iterations")
            extra = {}
    nthreads = max([u.get("num_threads", 1) for u in used] + [1])
    out = {"value": 1.0 / t_qp, "unit": "QP/s", "cores": int(nthreads), "kind": "oracle", "sample": sample,
           "seconds_per_qp": t_qp}
    out.update(extra)
    return out


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
    h = qpgpu.qp_create_from_problem(prob, settings=qpgpu.qp_default_settings(timing=1,
                                                                             spmv_format=args.spmv_format))
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
                      "format": ["csr", "line"][fmt], "spmv_schedule": info.get("spmv_schedule"),
                      "fwd_us": fus, "bwd_us": bus, "fwd_GBs": bf / fus / 1e3, "bwd_GBs": bb / bus / 1e3,
                      "fwd_bytes": bf, "bwd_bytes": bb,
                      "csr_equivalent_fwd_GBs": cf / fus / 1e3, "csr_equivalent_bwd_GBs": cb / bus / 1e3,
                      "checksum": float(np.abs(y).sum())}), flush=True)


def batch_run(probs, prec, steps, warmup):
    """`probs` created once at precision `prec` (qp_solve_batch's default
    mode: each QP's own solve, several in flight on their own streams), then
    solved together by qp_solve_batch `warmup` times untimed and `steps` times
    timed (host clock around the calls, data resident in HBM).  The handles
    are freed before returning."""
    from paper_2405_03584_amd import qpgpu
    t0 = time.perf_counter()
    st = qpgpu.qp_default_settings(precision=prec)
    hs = [qpgpu.qp_create_from_problem(p, settings=st) for p in probs]
    t_create = time.perf_counter() - t0
    print(f"[bench] batch {prec}: created {len(hs)} handles in {t_create:.1f}s", file=sys.stderr, flush=True)
    for i in range(warmup):
        s, _, infos = qpgpu.qp_solve_batch(hs)
        print(f"[bench] batch {prec} warmup {i}: status={s}", file=sys.stderr, flush=True)
    infos_all = []
    t0 = time.perf_counter()
    for i in range(steps):
        s, _, infos = qpgpu.qp_solve_batch(hs)
        infos_all += infos
    el = time.perf_counter() - t0
    for h in hs:
        h.close()
    ms = 1e3 * el / steps
    pcg = sum(f["pcg_iters"] for f in infos_all) / steps
    print(f"[bench] batch {prec}: {ms:.1f} ms per batch, pcg {pcg:.0f}", file=sys.stderr, flush=True)
    return {"ms_per_batch": ms, "qp_per_s": len(probs) / (ms * 1e-3),
            "status_ok": all(f["status"] == qpgpu.QP_OK for f in infos_all),
            "ipm_iters_total": sum(f["ipm_iters"] for f in infos_all) // steps,
            "pcg_phase_ms": max(f["t_pcg_ms"] for f in infos_all),   # per call: the batched directions
            "pcg_iters_total": int(pcg), "create_s": t_create,
            "max_certificate": max(max(f[k] for k in ("eps_d", "eps_p", "eps_c", "gap")) for f in infos_all)}


def batch_bench(args):
    """The uneven batch: `count` members of the 64-QP set, created once, then
    solved together (qp_solve_batch, --batch-mode 0: host workers, the
    default; 1: the persistent batched path) per step; for comparison the
    same QPs solved one after another, and in the other batch mode (its own
    handles)."""
    import qpsynth
    from paper_2405_03584_amd import qpgpu
    t0 = time.perf_counter()
    probs = [qpsynth.config4_instance(i) for i in range(args.count)]
    nnz = sum(int(p.J.nnz) for p in probs)
    print(f"[bench] generated {len(probs)} QPs, n in [{min(p.n for p in probs)}, {max(p.n for p in probs)}], "
          f"{nnz} nnz of J in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)

    def make(mode):
        st = qpgpu.qp_default_settings(precision=args.precision, graphs=args.graphs, batch_mode=mode)
        return [qpgpu.qp_create_from_problem(p, settings=st) for p in probs]

    hs = make(args.batch_mode)
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
    seq = other = None
    if args.compare:
        # the same handles solved one after another (one stream busy at a time)
        t1 = time.perf_counter()
        for h in hs:
            qpgpu.qp_solve(h)
        seq = time.perf_counter() - t1
        print(f"[bench] sequential: {1e3 * seq:.1f} ms", file=sys.stderr, flush=True)
        # the same batch in the other mode
        ho = make(1 - args.batch_mode)
        qpgpu.qp_solve_batch(ho)
        t2 = time.perf_counter()
        qpgpu.qp_solve_batch(ho)
        other = time.perf_counter() - t2
        for h in ho:
            h.close()
        print(f"[bench] batch mode {1 - args.batch_mode}: {1e3 * other:.1f} ms", file=sys.stderr, flush=True)
    modes = ["host workers", "persistent batched launches"]
    print(json.dumps({"metric": METRIC, "value": args.count * args.steps / el, "unit": "QP/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": args.precision, "data": "synthetic",
                      "config": {"workload": f"batch of {args.count} uneven banded-dose QPs "
                                             f"(n in [2000, 20000], {nnz} nnz of J in all), "
                                             f"{modes[args.batch_mode]}",
                                 "precision": args.precision, "batch_mode": args.batch_mode},
                      "status_ok": ok,
                      "sequential_ms": 1e3 * seq if seq else None,
                      "other_mode_ms": 1e3 * other if other else None,
                      "batch_speedup_vs_sequential": seq / (el / args.steps) if seq else None,
                      "batch_speedup_vs_other_mode": other / (el / args.steps) if other else None,
                      "ipm_iters_total": sum(f["ipm_iters"] for f in all_infos),
                      "pcg_iters_total": sum(f["pcg_iters"] for f in all_infos),
                      "pcg_phase_ms": max(f["t_pcg_ms"] for f in all_infos)}), flush=True)


def systems_bench(args):
    """The PCG systems and preconditioners on one QP (--systems-qp): the
    condensed system with the constraint-block preconditioner (the default),
    the condensed system with the paper's Jacobi preconditioner, and the
    paper's doubly augmented system (eq. (2x2_augmented), Jacobi).  The
    Jacobi variants are bounded (--pcg-cap PCG iterations per solve, 60 IPM
    iterations), since they stall once rows of A become active.  One solve
    each, FP64, data resident in HBM."""
    import qpsynth
    from paper_2405_03584_amd import qpgpu
    prob = qpsynth.config5(scale=args.scale) if args.systems_qp == "config5" else qpsynth.config2(scale=args.scale)
    runs = [("condensed, constraint block", {}),
            ("condensed, Jacobi", {"precond": 0, "pcg_max_iter": args.pcg_cap, "max_ipm_iter": 60}),
            ("doubly augmented, Jacobi", {"kkt_system": 1, "pcg_max_iter": args.pcg_cap, "max_ipm_iter": 60})]
    out = []
    for name, kw in runs:
        h = qpgpu.qp_create_from_problem(prob, settings=qpgpu.qp_default_settings(**kw))
        t0 = time.perf_counter()
        r = qpgpu.qp_solve(h)
        ms = 1e3 * (time.perf_counter() - t0)
        i = r.info
        rec = {"system": name, "status": r.status, "ipm_iters": i["ipm_iters"], "pcg_iters": i["pcg_iters"],
               "directions_at_pcg_cap": i["pcg_capped"], "ms": ms, "pcg_phase_ms": i["t_pcg_ms"],
               "us_per_pcg_iter": 1e3 * i["t_pcg_ms"] / max(i["pcg_iters"], 1), "mu": i["mu"],
               "rnorm": i["rnorm"], "objective": i["objective"]}
        print(f"[bench] {name}: status {r.status} ipm {i['ipm_iters']} pcg {i['pcg_iters']} {ms:.0f} ms",
              file=sys.stderr, flush=True)
        out.append(rec)
        h.close()
    print(json.dumps({"workload": f"PCG systems on the {args.systems_qp} QP (scale {args.scale})",
                      "pcg_cap": args.pcg_cap, "runs": out}), flush=True)


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
    ap.add_argument("--cpu-baseline", default="full", choices=["full", "sample", "none"],
                    help="full: the whole oracle solve on the host cores (about 2 minutes at n=20,000); "
                         "sample: dense H + one IPM iteration, extrapolated; none")
    ap.add_argument("--mixed", type=int, default=1, choices=[0, 1],
                    help="1: also time the other two precisions on the same QP")
    ap.add_argument("--batch", type=int, default=1, choices=[0, 1],
                    help="1: also time the 64-QP batch (qp_solve_batch) in each precision")
    ap.add_argument("--csr", type=int, default=1, choices=[0, 1],
                    help="1: also time the general CSR operator path on the same QP")
    ap.add_argument("--log", type=int, default=0, help="per-IPM-iteration progress on stderr (untimed runs)")
    ap.add_argument("--mode", default="solve", choices=["solve", "operator", "copy", "stream"],
                    help="solve: whole QP solves (the benchmark); operator: repeated operator "
                         "products only (for counter runs); copy: a plain device copy of the "
                         "J value+index bytes (counter calibration)")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--spmv-format", type=int, default=0, choices=[0, 1],
                    help="--mode operator: 0 the line format where J has it (the default), 1 CSR")
    ap.add_argument("--graphs", type=int, default=1, choices=[0, 1],
                    help="1: PCG iterations replayed as captured HIP graphs (the production setting); "
                         "0: direct launches (for kernel-trace and counter runs)")
    ap.add_argument("--workload", default="config2", choices=["config2", "config5", "batch", "sqp", "systems"],
                    help="config2: banded-dose QP n=20,000 (default, the benchmark line); config5: "
                         "n=60,000, BF16-valued J with 200M nnz and a rank-20 term; batch: the 64 "
                         "uneven QPs (n in [2000, 20000]) solved together by qp_solve_batch")
    ap.add_argument("--count", type=int, default=64, help="batch size for --workload batch")
    ap.add_argument("--systems-qp", default="config2", choices=["config2", "config5"],
                    help="--workload systems: the QP the PCG systems are compared on")
    ap.add_argument("--pcg-cap", type=int, default=3000,
                    help="--workload systems: PCG iterations per solve for the Jacobi variants")
    ap.add_argument("--compare", type=int, default=1, choices=[0, 1],
                    help="--workload batch: also time the QPs one at a time and in the other batch mode")
    ap.add_argument("--batch-mode", type=int, default=0, choices=[0, 1],
                    help="--workload batch: 0 host workers (the default of qp_solve_batch), 1 the "
                         "persistent batched path")
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
    if args.workload == "systems":
        return systems_bench(args)
    ceiling = stream_ceiling() if args.mode == "solve" else None   # before this process touches the GPU
    t0 = time.perf_counter()
    prob = qpsynth.config5(scale=args.scale) if args.workload == "config5" else qpsynth.config2(scale=args.scale)
    if args.mode == "operator":
        return operator_only(args, prob)
    n, m, nJ = prob.n, prob.m, prob.J.shape[0]
    nnzJ, nnzA = int(prob.J.nnz), int(prob.A.nnz)
    print(f"[bench] generated n={n} nJ={nJ} nnzJ={nnzJ} m={m} nnzA={nnzA} in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    gold = None
    gpath = os.path.join(ROOT, "tests", "golden", "config2_oracle.json")
    if args.workload == "config2" and args.scale == 1.0 and os.path.exists(gpath):
        gold = json.load(open(gpath))

    # The headline precision first, then the other two on the same QP (the
    # metric compares mixed precision with FP64).  Timed solves use the
    # production settings: captured PCG graphs, no per-kernel events, no log.
    precs = [args.precision] + ([q for q in ("bf16", "fp32", "fp64") if q != args.precision]
                                if args.mixed else [])
    runs = {}
    for prec in precs:
        runs[prec] = time_solves(args, prob, prec, gold)
    head = runs[args.precision]

    # Roofline: one more solve per precision on a handle with timing = 1 (HIP
    # events around each operator kernel on the library's stream).
    vbytes = {"fp64": 8, "fp32": 4, "bf16": 2}
    kern = {}
    for prec in precs:
        kern[prec] = kernel_rates(prob, prec, vbytes[prec])
    k0 = kern[args.precision]
    dom = k0["dominant"]
    csr = csr_operator_rates(prob, args.precision, vbytes[args.precision]) if args.csr else None

    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "QP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_qp"],
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
        "time_to_solution_ms": head["ms_per_qp"],
        "ipm_iters": head["ipm_iters"],
        "pcg_iters_per_qp": head["pcg_iters_per_qp"],
        "pcg_iters_per_s": head["pcg_iters_per_s"],
        "status_ok": head["status_ok"],
        "by_precision": {q: {**runs[q], "line_pass": kern[q]["line"], "spot_pass": kern[q]["spot"]}
                         for q in precs},
        "spmv": {"format": k0["format"], **k0["detail"]},
        "roofline": {"bound": "hbm", "kernel": dom["name"], "achieved": dom["GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dom["GBs"] / HBM_PEAK_GBS,
                     "traffic": (counter_traffic(dom["name"].split()[0], args.precision)
                                 if args.scale == 1.0 and args.workload == "config2" else None),
                     "bytes_per_launch": dom["bytes"], "avg_launch_us": dom["us"],
                     "stream_read_ceiling_GBs": ceiling,
                     "frac_of_stream_ceiling": dom["GBs"] / ceiling if ceiling else None},
        "csr_operator": csr,
        "create_s": head["create_s"],
    }
    if args.mixed and "fp64" in runs:
        out["mixed_vs_fp64"] = {q: runs["fp64"]["ms_per_qp"] / runs[q]["ms_per_qp"] for q in precs if q != "fp64"}
    if args.batch and args.workload == "config2":
        # the 64 uneven QPs (n in [2000, 20000]) solved together, per precision
        t0 = time.perf_counter()
        probs = [qpsynth.config4_instance(i) for i in range(64)]
        bnnz = sum(int(p.J.nnz) for p in probs)
        print(f"[bench] batch: generated 64 QPs ({bnnz} nnz of J) in {time.perf_counter() - t0:.1f}s",
              file=sys.stderr, flush=True)
        bruns = {q: batch_run(probs, q, 1, 1) for q in ("fp64", "bf16", "fp32")}
        del probs
        out["batch64"] = {"workload": f"64 uneven banded-dose QPs, n in [2000, 20000], {bnnz} nnz of J in all, "
                                      "one qp_solve_batch (default mode: host workers) per step",
                          "by_precision": bruns,
                          "mixed_vs_fp64": {q: bruns["fp64"]["ms_per_batch"] / bruns[q]["ms_per_batch"]
                                            for q in ("bf16", "fp32")}}
    # the paper's speedups are over a commercial CPU solver on its own clinical
    # QPs and machines: printed beside ours for context, not compared
    out["paper_context"] = {
        "speedup_over_raystation_qp_solver": {"proton_head_and_neck_200_qps": 4.4,
                                              "vmat_head_and_neck_33_qps": 1.4},
        "paper_hardware": "paper's solver on an RTX 4080 GPU with a Ryzen 9 7900X host; RayStation 2024A "
                          "on an Intel i9-7940X",
        "precision": "FP64"}
    if args.cpu_baseline != "none" and args.workload == "config2":
        print(f"[bench] cpu baseline ({args.cpu_baseline} oracle)...", file=sys.stderr, flush=True)
        iters = gold["ipm_iters"] if gold else head["ipm_iters"]
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_baseline, iters)
        out["speedup_over_cpu_oracle"] = out["value"] / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


def time_solves(args, prob, prec, gold):
    """Whole solves of one QP at one precision: `warmup` untimed, `steps`
    timed back to back (host clock around the calls, data resident in HBM)."""
    from paper_2405_03584_amd import qpgpu
    settings = qpgpu.qp_default_settings(precision=prec, log_level=args.log, graphs=args.graphs)
    t0 = time.perf_counter()
    h = qpgpu.qp_create_from_problem(prob, settings=settings)
    t_create = time.perf_counter() - t0
    print(f"[bench] {prec}: qp_create {t_create:.2f}s", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        r = qpgpu.qp_solve(h)
        print(f"[bench] {prec} warmup {i}: status={r.status} ipm={r.info['ipm_iters']} "
              f"pcg={r.info['pcg_iters']} {r.info['t_solve_ms']:.1f} ms", file=sys.stderr, flush=True)
    infos = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = qpgpu.qp_solve(h)
        infos.append(r.info)
    elapsed = time.perf_counter() - t0
    h.close()
    pcg = sum(i["pcg_iters"] for i in infos)
    pcg_ms = sum(i["t_pcg_ms"] for i in infos)
    out = {"value": args.steps / elapsed, "ms_per_qp": 1e3 * elapsed / args.steps,
           "ipm_iters": infos[-1]["ipm_iters"], "pcg_iters_per_qp": pcg / args.steps,
           "pcg_iters_per_s": pcg / (pcg_ms * 1e-3) if pcg_ms > 0 else None,
           "status_ok": all(i["status"] == qpgpu.QP_OK for i in infos),
           "prec_fallbacks": sum(i["prec_fallbacks"] for i in infos),
           "certificate": max(infos[-1][k] for k in ("eps_d", "eps_p", "eps_c", "gap")),
           "create_s": t_create}
    if gold is not None:
        out["parity"] = {"x_max_abs_err_vs_oracle": float(np.abs(r.x - np.array(gold["x"])).max()),
                         "objective_rel_err_vs_oracle": abs(infos[-1]["objective"] - gold["objective"])
                         / abs(gold["objective"])}
    print(f"[bench] {prec}: {out['ms_per_qp']:.1f} ms per QP, ipm {out['ipm_iters']}, "
          f"pcg {out['pcg_iters_per_qp']:.0f}", file=sys.stderr, flush=True)
    return out


def kernel_rates(prob, prec, vb):
    """Per-launch duration of the operator kernels over a whole solve on a
    handle with timing = 1 (direct launches, HIP events on the library's
    stream; launches past a converged PCG solve excluded), and their
    algorithmic GB/s."""
    from paper_2405_03584_amd import qpgpu
    n, m, nJ = prob.n, prob.m, prob.J.shape[0]
    nnzJ, nnzA = int(prob.J.nnz), int(prob.A.nnz)
    ht = qpgpu.qp_create_from_problem(prob, settings=qpgpu.qp_default_settings(precision=prec, timing=1))
    rt = qpgpu.qp_solve(ht)
    ht.close()
    i = rt.info
    fmt = i["spmv_format"]
    bf, bb = spmv_bytes(n, nJ, m, nnzJ, nnzA, vb, fmt)
    cf, cb = spmv_bytes(n, nJ, m, nnzJ, nnzA, vb, 0)
    fus = 1e3 * i["t_spmv_fwd_ms"] / max(i["n_spmv_fwd"], 1)
    bus = 1e3 * i["t_spmv_bwd_ms"] / max(i["n_spmv_bwd"], 1)
    if fmt == 1:
        names = ("k_line_pass (J p, W scaling and per-slot J^T contributions from one read of J; u from A z and A p)",
                 "k_spot_pass (per-spot J^T sums, A^T u, epilogue and p.q partials)")
    else:
        names = ("k_op_fwd (J + A SpMV, fused W / Sigma_A scaling)",
                 "k_op_bwd (J^T + A^T SpMV, fused epilogue and p.q partials)")
    fwd = {"name": names[0], "bytes": bf, "us": fus, "GBs": bf / (fus * 1e-6) / 1e9}
    bwd = {"name": names[1], "bytes": bb, "us": bus, "GBs": bb / (bus * 1e-6) / 1e9}
    print(f"[bench] {prec} kernels: {names[0].split()[0]} {fus:.1f} us ({fwd['GBs']:.0f} GB/s), "
          f"{names[1].split()[0]} {bus:.1f} us", file=sys.stderr, flush=True)
    return {"format": ["csr", "line"][fmt], "line": fwd, "spot": bwd,
            "dominant": bwd if bus >= fus else fwd,
            "detail": {"fwd_us": fus, "bwd_us": bus, "fwd_GBs": fwd["GBs"], "bwd_GBs": bwd["GBs"],
                       "fwd_bytes": bf, "bwd_bytes": bb, "timed_launches": i["n_spmv_bwd"],
                       "csr_equivalent_fwd_GBs": cf / (fus * 1e-6) / 1e9,
                       "csr_equivalent_bwd_GBs": cb / (bus * 1e-6) / 1e9}}


def csr_operator_rates(prob, prec, vb, reps=20):
    """The same QP's operator on the general CSR path (spmv_format = 1: J and
    the stored J^T, each pass reading values and column indices): per-launch
    time of each pass over `reps` products and its algorithmic GB/s."""
    from paper_2405_03584_amd import qpgpu
    import qpsynth
    it = qpsynth.random_iterate(prob, 1)
    h = qpgpu.qp_create_from_problem(prob, settings=qpgpu.qp_default_settings(timing=1, spmv_format=1))
    _, info = qpgpu.qp_operator_apply(h, it["sigma_x"], it["sigma_A"], it["v"], precision=prec, reps=reps)
    h.close()
    n, m, nJ = prob.n, prob.m, prob.J.shape[0]
    bf, bb = spmv_bytes(n, nJ, m, int(prob.J.nnz), int(prob.A.nnz), vb, 0)
    fus = 1e3 * info["t_spmv_fwd_ms"] / max(info["n_spmv_fwd"], 1)
    bus = 1e3 * info["t_spmv_bwd_ms"] / max(info["n_spmv_bwd"], 1)
    sched = info["spmv_schedule"]
    out = {"precision": prec, "reps": reps, "schedule": sched,
           "J_pass": {"kernel": "k_op_fwd_stream" if sched == 1 else f"k_op_fwd<{sched}>", "us": fus, "bytes": bf,
                      "GBs": bf / (fus * 1e-6) / 1e9,
                      "frac": bf / (fus * 1e-6) / 1e9 / HBM_PEAK_GBS},
           "Jt_pass": {"kernel": "k_op_bwd", "us": bus, "bytes": bb, "GBs": bb / (bus * 1e-6) / 1e9,
                       "frac": bb / (bus * 1e-6) / 1e9 / HBM_PEAK_GBS}}
    print(f"[bench] CSR operator {prec} (schedule {sched}): J pass {fus:.1f} us ({out['J_pass']['GBs']:.0f} GB/s), "
          f"J^T pass {bus:.1f} us ({out['Jt_pass']['GBs']:.0f} GB/s)", file=sys.stderr, flush=True)
    return out


if __name__ == "__main__":
    main()
