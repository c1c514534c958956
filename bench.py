#!/usr/bin/env python3
"""Throughput of the Sparse Frequent Directions hot path on one MI355X.

One step = one pass of the whole path over the workload: reset the handle, append every row
(CSR already resident in HBM; each full buffer goes through the buffer step: CSC build,
SimultaneousIteration, VerifySpectral, BoostedSparseShrink, DenseShrink) and query the sketch.

Workload of the line's value: n = 1,000,000 rows, d = 100,000, Poisson(50) entries per row from
Zipf(1.0) columns, lognormal(0,1) values plus a planted rank-20 component with 30% of the energy,
ell = 50, eps = 1/4, FP32 (workloads.stream_1e6_d1e5).

Prints one JSON line: the metric, its value in nnz/s, the roofline of the dominant kernel class
(HIP events on the library's stream), the FP64 oracle's rate on a bounded sample of the same
stream (cpu_baseline), and under "forms" the forms the metric compares, each timed in the same
run: the BF16 precision form on the same stream, the 2e6-row d = 5e4 stream at ell = 200 and the
1e7-row d = 1e6 stream at ell = 100 (both generated on the device) in FP32 and BF16, and the
batched form on all 4,096 streams of the batching workload, with each form's covariance error
(Sec. 4) from the FP64 evaluator.

Only the cpu_baseline leg (the functions named cpu_baseline*) runs the FP64 oracle.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "ingested nnz/s on 1 MI355X at fixed cov-err; BF16/batched vs plain FP32"
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFS = 157.3
HERE = os.path.dirname(os.path.abspath(__file__))
# options of the timed handles (--autotune, --graphs)
SKETCH_OPTS: dict = {}
BATCH_OPTS: dict = {}

# HBM traffic of one product measured with rocprofv3 --pmc (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0
# per dispatch, the factors that make a plain 1 GiB copy read as 1 GiB each way), summed over the
# product's kernels.  Valid only for the workload, panel precision and kernel sources it was taken
# with (sha256 prefix of the sources, concatenated in the order listed).
TRAFFIC_SOURCES = ("paper_1602_00412_amd/csrc/sfd_spmm.hip", "paper_1602_00412_amd/csrc/sfd_internal.h")
MEASURED_TRAFFIC = {
    # (class, workload, precision): (bytes per call, sha256 prefix of TRAFFIC_SOURCES, summary)
    ("spmm_csc", "stream1e6", "fp32"): (6.4540e+08, "f20bfb611243cd82",
                                      "profiles/sfd_spmm_csc_ell50_1e5row_buffers_hbm_traffic.txt"),
}


def traffic_sources_sha() -> str:
    import hashlib

    h = hashlib.sha256()
    for src in TRAFFIC_SOURCES:
        with open(os.path.join(HERE, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(cls: str, workload: str, precision: str):
    ent = MEASURED_TRAFFIC.get((cls, workload, precision))
    if not ent:
        return None
    nbytes, sha, _ = ent
    try:
        cur = traffic_sources_sha()
    except OSError:
        return None
    return nbytes if cur.startswith(sha) else None


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gram_rel_distance(B1, B2) -> float:
    """||B1^T B1 - B2^T B2||_F / ||B2^T B2||_F in FP64 from the small Grams (the sketches' d x d
    covariances are never formed): ||X^T X||_F^2 = ||X X^T||_F^2 and <B1^T B1, B2^T B2> =
    ||B1 B2^T||_F^2."""
    import numpy as np

    B1 = np.asarray(B1, dtype=np.float64)
    B2 = np.asarray(B2, dtype=np.float64)
    a = np.sum((B1 @ B1.T) ** 2)
    c = np.sum((B2 @ B2.T) ** 2)
    x = np.sum((B1 @ B2.T) ** 2)
    return float(np.sqrt(max(a + c - 2.0 * x, 0.0) / c)) if c > 0 else float(np.sqrt(a))


def free_gpu():
    import gc

    import torch

    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def cpu_baseline(st, ell: int, rows: int):
    """The FP64 oracle on the first `rows` rows of the stream (query folds them in one buffer)."""
    import numpy as np

    from oracle import SFDOracle

    try:
        from threadpoolctl import threadpool_info

        threads = max([int(p.get("num_threads", 1)) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    sub = st.rows(0, rows)
    t0 = time.perf_counter()
    o = SFDOracle(st.d, ell, 0.25, 0)
    o.append_csr(sub.indptr, sub.indices, sub.values)
    rec = []
    B, _, _ = o.query(log=rec)
    dt = time.perf_counter() - t0
    qs = sorted({r["q"] for b in o.log for r in b["attempts"]} | {r["q"] for r in rec})
    return sub, B.astype(np.float64), {
        "value": sub.nnz / dt,
        "unit": "nnz/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {rows} rows ({sub.nnz} nnz) of the same stream, folded by one query "
                  f"({o.flushes} flushes + the query's fold; q={','.join(map(str, qs)) or 'none'}); {dt:.1f} s; "
                  f"BLAS threads={threads}, scipy sparse products single-threaded",
    }


def cpu_baseline_eval_refs(sub, Bg, k: int = 10):
    """The oracle evaluator's measures of a GPU sketch Bg of the sample sub (the references of the
    GPU evaluator's check): ||A||_F^2 and proj-err (k) by their definitions (Sec. 4)."""
    from oracle import evaluate

    A = sub.to_scipy()
    return evaluate.fro2(A), evaluate.proj_err(A, Bg, k)


def cpu_baseline_prefix(st, ell: int, q: int):
    """The FP64 oracle's sketch of a prefix st with a fixed q (the device path's parity check on
    the large workloads, where the oracle's d x ell Householder QRs at the method's q would take
    minutes); returns (sketch, seconds)."""
    from oracle import SFDOracle

    t = time.perf_counter()
    o = SFDOracle(st.d, ell, 0.25, 0, q=q, unit_roundoff=2.0 ** -24)
    o.append_csr(st.indptr, st.indices, st.values)
    return o.sketch(), time.perf_counter() - t


def cpu_baseline_stream(indptr, indices, values, d: int, ell: int, stream_id: int):
    """The FP64 oracle on one whole stream of a batch (host arrays): (sketch, nnz/s, seconds)."""
    from oracle import SFDOracle

    t = time.perf_counter()
    o = SFDOracle(d, ell, 0.25, 0, stream_id=stream_id, unit_roundoff=2.0 ** -24)
    o.append_csr(indptr, indices, values)
    B = o.sketch()
    dt = time.perf_counter() - t
    return B, (int(indptr[-1] - indptr[0]) / dt if dt > 0 else None), dt


def measure_batch_full(streams: int, steps: int, warmup: int) -> dict:
    """The batched form on streams 0 .. streams - 1 of the batching workload (d = 2e4, ell = 32,
    Poisson(30) entries per row, Zipf(1.1) columns, lognormal(0,1) values, 1e3..1e5 rows per
    stream), generated on the device, resident in HBM, appended in one batch call and queried.
    Checks: streams 0, 1 and the shortest equal bit for bit to single-stream handles; the shortest
    against the FP64 oracle (cpu_baseline leg, which also times it)."""
    import numpy as np
    import torch

    from paper_1602_00412_amd import sfd
    from workloads.device import batch_streams_d2e4

    t0 = time.perf_counter()
    ptr, idx, val, starts = batch_streams_d2e4("cuda", streams=streams)
    torch.cuda.synchronize()
    S, d, ell = len(starts) - 1, 20_000, 32
    nnz = int(ptr[-1].item())
    log(f"batch: generated {S} streams, {starts[-1]} rows, {nnz} nnz in {time.perf_counter() - t0:.1f} s")
    bat = sfd.Batch(S, d, ell, **BATCH_OPTS)
    b_out = torch.empty((S, ell, d), dtype=torch.float32, device="cuda")
    sos = np.arange(S, dtype=np.int32)

    def step():
        bat.reset()
        bat.append_csr(sos, starts, ptr, idx, val)
        bat.sketch(out=b_out)

    for w in range(warmup):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"batch warmup {w + 1}/{warmup}: {time.perf_counter() - t:.3f} s")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(steps):
        step()
        log(f"batch step {k + 1}/{steps} done")
    torch.cuda.synchronize()
    el = (time.perf_counter() - t) / steps
    flushes = sum(bat.stats(s)["flushes"] for s in range(S))
    log(f"batch: {1e3 * el:.1f} ms/step, {nnz / el:.3e} nnz/s, {flushes} buffer steps")
    lens = np.diff(starts)
    short = int(np.argmin(lens))
    bitwise = True
    for s_ in sorted({0, 1, short}):
        one = sfd.Sketch(d, ell, 0.25, 0, stream_id=s_)
        lo, hi = int(starts[s_]), int(starts[s_ + 1])
        one.append_csr(ptr[lo:hi + 1], idx, val)
        bitwise = bitwise and torch.equal(one.sketch(), b_out[s_])
        one.close()
    lo, hi = int(starts[short]), int(starts[short + 1])
    a, b = int(ptr[lo].item()), int(ptr[hi].item())
    Bo, rate, dt = cpu_baseline_stream((ptr[lo:hi + 1] - a).cpu().numpy(), idx[a:b].cpu().numpy(),
                                       val[a:b].cpu().numpy(), d, ell, short)
    parity = gram_rel_distance(b_out[short].cpu().numpy(), Bo)
    log(f"batch samples: bitwise equal to single-stream handles: {bitwise}; stream {short} ({hi - lo} rows) vs "
        f"oracle {parity:.2e}")
    rec = {"value": nnz / el, "unit": "nnz/s", "ms_per_step": 1e3 * el, "steps": steps, "warmup": warmup,
           "streams": S, "rows": int(starts[-1]), "nnz": nnz, "d": d, "ell": ell, "buffers_per_step": flushes,
           "bitwise_equal_to_single_stream": bool(bitwise), "oracle_stream": short,
           "oracle_rel_frobenius": parity,
           "cpu_baseline": {"value": rate, "unit": "nnz/s", "kind": "oracle",
                            "sample": f"stream {short} ({hi - lo} rows, {b - a} nnz), whole; {dt:.1f} s"}}
    bat.close()
    del ptr, idx, val, b_out
    free_gpu()
    return rec


FORM_QUEUES = {"ell200": 32, "d1e6": 16, "batch4096": 16}  # hardware queues of each form's process


def run_form_child(name: str, args) -> dict:
    """One form measured by a child process (bench.py --form-child name), its record parsed from
    the JSON line it prints."""
    import subprocess

    if name not in FORM_QUEUES:
        raise SystemExit(f"unknown form {name}")
    env = dict(os.environ)
    env["GPU_MAX_HW_QUEUES"] = str(FORM_QUEUES[name])
    cmd = [sys.executable, os.path.abspath(__file__), "--form-child", name, "--autotune", str(args.autotune),
           "--graphs", str(args.graphs), "--launch", args.launch]
    log(f"form {name}: child process, {FORM_QUEUES[name]} hardware queues")
    res = subprocess.run(cmd, env=env, stdout=subprocess.PIPE, text=True)
    if res.returncode != 0:
        raise SystemExit(f"form {name} failed (exit {res.returncode})")
    return json.loads(res.stdout.strip().splitlines()[-1])


def form_child(name: str) -> int:
    """The child side of run_form_child: measures one form and prints its record."""
    if name in ("ell200", "d1e6"):
        rec = measure_large_stream(name, 1, 1)
    else:
        rec = measure_batch_full(4096, 1, 1)
    print(json.dumps(rec), flush=True)
    return 0


def run_batch_full(args) -> int:
    """All 4,096 streams of the batching workload as the line's workload."""
    rec = measure_batch_full(args.batch_first_streams, args.steps, args.warmup)
    line = {
        "metric": METRIC, "value": rec["value"], "unit": "nnz/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": rec["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{rec['streams']} independent zipf-poisson streams, {rec['rows']} rows, d=20000, "
                               f"lambda=30, s=1.1, lognormal, ell=32 eps=1/4, generated on the device, one batch call",
                   "nnz": rec["nnz"], "ell": 32, "buffers_per_step": rec["buffers_per_step"],
                   "parallelism": "1 GPU"},
        "roofline": None, "cpu_baseline": rec["cpu_baseline"],
        "samples": {k: rec[k] for k in ("bitwise_equal_to_single_stream", "oracle_stream", "oracle_rel_frobenius")},
    }
    print(json.dumps(line), flush=True)
    return 0


def measure_large_stream(which: str, steps: int, warmup: int, check_rows: int = 2000) -> dict:
    """A stream generated on the device in both forms: which = "ell200" (2e6 rows, d = 5e4,
    Poisson(80), Zipf(1.1), N(0,1) + planted rank-50, ell = 200) or "d1e6" (1e7 rows, d = 1e6,
    Poisson(100), Zipf(1.0), lognormal + planted rank-100 at 30% energy, ell = 100).  FP32 and
    BF16 are timed one after the other on the same resident stream (same q, same random blocks);
    cov-err of each sketch from the FP64 evaluator (sfd_evaluate) against the whole stream; parity
    of the FP32 path with the oracle on a check_rows prefix at q = 3 (cpu_baseline leg)."""
    import numpy as np
    import torch

    from paper_1602_00412_amd import sfd
    from workloads.device import stream_1e7_d1e6, stream_2e6_d5e4

    big = which == "d1e6"
    d, ell = (1_000_000, 100) if big else (50_000, 200)
    t0 = time.perf_counter()
    indptr, indices, values = (stream_1e7_d1e6 if big else stream_2e6_d5e4)("cuda")
    torch.cuda.synchronize()
    n, nnz = indptr.numel() - 1, int(indptr[-1].item())
    log(f"{which}: generated n={n} d={d} nnz={nnz} in {time.perf_counter() - t0:.1f} s")
    rec = {"rows": n, "d": d, "ell": ell, "nnz": nnz, "steps": steps, "warmup": warmup}
    out = torch.empty((ell, d), dtype=torch.float32, device="cuda")
    for prec in ("fp32", "bf16"):
        sk = sfd.Sketch(d, ell, 0.25, 0, precision=prec, **SKETCH_OPTS)

        def step():
            sk.reset()
            sk.append_csr(indptr, indices, values)
            sk.sketch(out=out)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t) / steps
        r = {"value": nnz / el, "unit": "nnz/s", "ms_per_step": 1e3 * el, "buffers_per_step": sk.stats()["flushes"],
             "q_last": sk.stats()["last_q"]}
        t = time.perf_counter()
        ev = sfd.evaluate(indptr, indices, values, d, out, k=0, steps=160)
        r["cov_err"] = ev["cov_err"]
        r["cov_max_ritz_residual"] = ev["cov_max_res"]
        r["eval_seconds"] = time.perf_counter() - t
        rec[prec] = r
        log(f"{which} {prec}: {1e3 * el:.1f} ms/step, {nnz / el:.3e} nnz/s, cov-err {ev['cov_err']:.4e}")
        sk.close()
        free_gpu()
    rec["bf16_speedup_vs_fp32"] = rec["fp32"]["ms_per_step"] / rec["bf16"]["ms_per_step"]
    rec["bf16_cov_err_over_fp32"] = rec["bf16"]["cov_err"] / rec["fp32"]["cov_err"]
    # parity of the FP32 path on a prefix (the same kernels and shapes, q shortened to 3)
    from workloads import CsrStream

    ppre = indptr[:check_rows + 1].cpu().numpy()
    st = CsrStream(ppre, indices[:int(ppre[-1])].cpu().numpy(), values[:int(ppre[-1])].cpu().numpy(), d,
                   dict(name=f"{which} prefix"))
    Bo, dt = cpu_baseline_prefix(st, ell, 3)
    sk2 = sfd.Sketch(d, ell, 0.25, 0, q=3)
    sk2.append_csr(torch.from_numpy(st.indptr).cuda(), torch.from_numpy(st.indices).cuda(),
                   torch.from_numpy(st.values).cuda())
    rec["prefix_parity_rel_frobenius"] = gram_rel_distance(sk2.sketch().cpu().numpy(), Bo)
    rec["prefix_parity_rows"] = check_rows
    sk2.close()
    log(f"{which}: bf16 {rec['bf16_speedup_vs_fp32']:.2f}x FP32 at cov-err {rec['bf16_cov_err_over_fp32']:.4f}x; "
        f"prefix parity ({check_rows} rows, q=3) {rec['prefix_parity_rel_frobenius']:.2e} ({dt:.1f} s oracle)")
    del indptr, indices, values, out
    free_gpu()
    return rec


def run_paper_sweep(args) -> int:
    """The paper's own synthetic workload (Sec. 4: rows of z distinct +-1 entries, 90% of them in the
    first 1.5 z columns) swept as in its Table 1: one parameter at a time over its range, the others
    at their defaults (n = 10,000, d = 1,000, ell = 50, z = 100): z in 5..500, d in 1e3..6e3, n in
    1e4..6e4, ell in 5..100.  Three algorithms on the GPU: SFD (Alg 2 with BoostedSparseShrink),
    SFD with SparseShrink alone (VerifySpectral off, as in the paper's experiments) and
    FrequentDirections (Sec. 2.1, DenseShrink of ell-row batches).  Reports ms per pass and the
    cov-err (Sec. 4, k = 10 for proj-err) of each sketch from the GPU evaluator; the paper reports
    SFD faster than FD on sparse inputs and not on dense ones."""
    import torch

    from paper_1602_00412_amd import sfd
    from workloads import paper_head_tail

    defaults = {"n": 10_000, "d": 1000, "z": 100, "ell": 50}
    sweeps = {"z": (5, 10, 20, 50, 100, 200, 500), "d": (1000, 2000, 4000, 6000),
              "n": (10_000, 20_000, 40_000, 60_000), "ell": (5, 10, 20, 50, 100)}
    algos = (("sfd", {}), ("sfd_noverify", {"verify": 0}), ("fd", {"algorithm": "fd"}))
    rows = []
    for param, values in sweeps.items():
        for v in values:
            p = dict(defaults, **{param: v})
            n, d, z, ell = p["n"], p["d"], p["z"], p["ell"]
            st = paper_head_tail(n=n, d=d, z=z)
            ptr = torch.from_numpy(st.indptr).cuda()
            idx = torch.from_numpy(st.indices).cuda()
            val = torch.from_numpy(st.values).cuda()
            out = torch.empty((ell, d), dtype=torch.float32, device="cuda")
            rec = {"sweep": param, "n": n, "d": d, "z": z, "ell": ell, "nnz": st.nnz}
            for name, opts in algos:
                sk = sfd.Sketch(d, ell, 0.25, 0, **opts)

                def step():
                    sk.reset()
                    sk.append_csr(ptr, idx, val)
                    sk.sketch(out=out)

                for _ in range(args.warmup):
                    step()
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(args.steps):
                    step()
                torch.cuda.synchronize()
                ms = 1e3 * (time.perf_counter() - t) / args.steps
                ev = sfd.evaluate(ptr, idx, val, d, out, k=min(10, ell), steps=min(d, 300))
                rec[name] = {"ms": ms, "cov_err": ev["cov_err"], "proj_err": ev["proj_err"],
                             "buffers": sk.stats()["flushes"]}
                sk.close()
            rec["fd_over_sfd_time"] = rec["fd"]["ms"] / rec["sfd_noverify"]["ms"]
            rows.append(rec)
            log(f"{param} sweep n={n} d={d} z={z} ell={ell}: sfd {rec['sfd']['ms']:.1f} ms, sfd w/o verify "
                f"{rec['sfd_noverify']['ms']:.1f} ms, fd {rec['fd']['ms']:.1f} ms; cov-err "
                f"{rec['sfd']['cov_err']:.4f} / {rec['sfd_noverify']['cov_err']:.4f} / {rec['fd']['cov_err']:.4f}")
    print(json.dumps({"workload": "paper head/tail generator (Sec. 4), Table 1 sweeps, eps=1/4",
                      "defaults": defaults, "steps": args.steps, "warmup": args.warmup, "points": rows}), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample-rows", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel-class pass (roofline, phases)")
    ap.add_argument("--profile-only", action="store_true",
                    help="warm-up and the per-kernel-class pass only (no timed steps; for rocprofv3 runs)")
    ap.add_argument("--rows", type=int, default=1_000_000, help="stream length (default: the full workload)")
    ap.add_argument("--csc-bands", type=int, default=0, choices=[0, 1, 8],
                    help="XCD-local pieces of the transposed products: 0 automatic, 1 off, 8 on")
    ap.add_argument("--csc-hot-min", type=int, default=0,
                    help="entries from which a CSC column is cut into XCD-local pieces (0: the library's default)")
    ap.add_argument("--no-forms", action="store_true", help="skip the BF16 and batched forms' timing")
    ap.add_argument("--form-steps", type=int, default=3, help="timed steps of the forms on the 10^6-row stream")
    ap.add_argument("--autotune", type=int, default=0, choices=[0, 1],
                    help="SFD_OPT_AUTOTUNE of every handle (0, the default: static product launches)")
    ap.add_argument("--launch", default="auto", choices=["auto", "static", "queue", "stage"],
                    help="SFD_OPT_PRODUCT_LAUNCH of the single-stream handles (auto: the tuned launch with --autotune 1, else the static grid)")
    ap.add_argument("--graphs", type=int, default=1, choices=[0, 1],
                    help="SFD_OPT_GRAPHS of the batch handles (1: graph-captured group steps, the default)")
    ap.add_argument("--big-forms", default="ell200,d1e6,batch4096",
                    help="forms on their own workloads timed after the line, each in a child process "
                         "(comma-separated; empty: none)")
    ap.add_argument("--form-child", default="", help=argparse.SUPPRESS)
    ap.add_argument("--batch-streams", type=int, default=64,
                    help="streams of the batched form (4,096-stream recipe: d=2e4, ell=32, Poisson(30)); 0 skips it")
    ap.add_argument("--lanes", type=int, default=0, help="lanes of the timed FP32 line (0: the library's default)")
    ap.add_argument("--hw-queues", type=int, default=0, choices=[0, 1, 2, 4, 8, 16, 32],
                    help="HIP hardware queues for this process (0: at least 16, 32 for the ell = 200 workload)")
    ap.add_argument("--precision", choices=["fp32", "bf16"], default="fp32",
                    help="panel precision of the main (timed and profiled) form; the line's value is FP32's")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--workload", choices=["stream1e6", "ell200", "d1e6", "batch4096", "paper"], default="stream1e6",
                    help="stream1e6: the 1e6-row stream at ell=50 (default); ell200: the 2e6-row, d=5e4 stream "
                         "at ell=200 (N(0,1) values), generated on the device, FP32 and BF16; "
                         "d1e6: the 1e7-row, d=1e6 stream "
                         "at ell=100, generated on the device, FP32 and BF16; batch4096: all 4,096 batch streams, "
                         "generated on the device, one batch call; paper: the paper's head/tail +-1 generator "
                         "swept over entries per row and over d, SFD (with and without VerifySpectral) "
                         "against FrequentDirections on the GPU")
    ap.add_argument("--batch-first-streams", type=int, default=4096, help="batch4096: the first this many streams")
    args = ap.parse_args()
    # HIP maps streams onto a per-process pool of hardware queues (4 by default) and streams
    # beyond it share queues: with 16 (32 when the handles run 8 lanes each), torch's stream and
    # the lane and main streams of both handles created here (FP32 line, BF16 form; or the
    # batch's 16 lanes) get queues of their own, so concurrent buffer steps do not serialise
    # behind one another.  Set before HIP starts; a larger value already in the environment is
    # kept.
    if args.hw_queues:
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    else:
        # the ell = 200 workload's handles run 8 lanes each (the forms run in child processes with
        # their own setting)
        want = 32 if args.workload == "ell200" else 16
        try:
            have = int(os.environ.get("GPU_MAX_HW_QUEUES", "0"))
        except ValueError:
            have = 0
        if have < want:
            os.environ["GPU_MAX_HW_QUEUES"] = str(want)
    SKETCH_OPTS.update(autotune=bool(args.autotune), graphs=bool(args.graphs), launch=args.launch)
    BATCH_OPTS.update(autotune=bool(args.autotune), graphs=bool(args.graphs))
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sketch shards by rows with "
              f"one merge at the end; runs across several GPUs are not implemented", file=sys.stderr)
        return 2

    # The forms on their own workloads (ell = 200; d = 1e6, ell = 100; all 4,096 batch streams):
    # each in a child process of its own with its own hardware-queue count, one after another,
    # before this process starts on the GPU (so no idle queues of this process compete with
    # theirs); the records join the line's "forms".
    big_forms = {}
    if (not args.form_child and not args.no_forms and not args.profile_only and not args.copy_probe_mib
            and args.precision == "fp32" and args.workload == "stream1e6"):
        for name in args.big_forms.split(","):
            name = name.strip()
            if name:
                big_forms[name] = run_form_child(name, args)

    import numpy as np
    import torch

    from paper_1602_00412_amd import sfd
    from workloads import stream_1e6_d1e5

    sfd.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.copy_probe_mib:
        # a copy of known size: its FETCH_SIZE / WRITE_SIZE readings calibrate the counters
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n, "launches": 3}), flush=True)
        return 0
    if args.form_child:
        return form_child(args.form_child)
    if args.workload == "batch4096":
        return run_batch_full(args)
    if args.workload == "paper":
        return run_paper_sweep(args)
    t0 = time.perf_counter()
    if args.workload in ("d1e6", "ell200"):
        from workloads.device import stream_2e6_d5e4, stream_1e7_d1e6
        from workloads import CsrStream

        big = args.workload == "d1e6"
        n_dev = args.rows if args.rows != 1_000_000 else (10_000_000 if big else 2_000_000)
        d_dev = 1_000_000 if big else 50_000
        indptr, indices, values = (stream_1e7_d1e6 if big else stream_2e6_d5e4)("cuda", n=n_dev)
        torch.cuda.synchronize()
        ell = 100 if big else 200
        # host copy of a prefix: the sample the oracle checks
        pre = min(args.cpu_sample_rows, n_dev)
        ppre = indptr[:pre + 1].cpu().numpy()
        st = CsrStream(ppre, indices[:int(ppre[-1])].cpu().numpy(), values[:int(ppre[-1])].cpu().numpy(),
                       d_dev, dict(name=f"{args.workload} prefix"))
        st_n, st_d, st_nnz = n_dev, d_dev, int(indptr[-1].item())
        if big:
            desc = (f"zipf-poisson stream n={st_n} d={st_d} lambda=100 s=1.0 lognormal+planted rank-100 (30%), "
                    f"ell={ell} eps=1/4, generated on the device")
        else:
            desc = (f"zipf-poisson stream n={st_n} d={st_d} lambda=80 s=1.1 N(0,1)+planted rank-50 (sigma_i=1/i), "
                    f"ell={ell} eps=1/4, generated on the device")
    else:
        st = stream_1e6_d1e5(seed=0, n=args.rows)
        ell = 50
        indptr = torch.from_numpy(st.indptr).cuda()
        indices = torch.from_numpy(st.indices).cuda()
        values = torch.from_numpy(st.values).cuda()
        st_n, st_d, st_nnz = st.n, st.d, st.nnz
        desc = f"zipf-poisson stream n={st.n} d={st.d} lambda=50 s=1.0 lognormal+planted rank-20 (30%), ell={ell} eps=1/4"
    log(f"generated n={st_n} d={st_d} nnz={st_nnz} in {time.perf_counter() - t0:.1f} s")
    out = torch.empty((ell, st_d), dtype=torch.float32, device="cuda")
    sk = sfd.Sketch(st_d, ell, 0.25, 0, csc_bands=args.csc_bands or None, csc_hot_min=args.csc_hot_min or None,
                    **SKETCH_OPTS,
                    precision=args.precision)
    if args.lanes:
        sk.set_option(sfd.OPT_LANES, args.lanes)
    lanes_main = args.lanes or (8 if ell > 128 else 4)  # the library's default lanes
    Lw_main = 32 if ell <= 32 else 64 if ell <= 64 else 128 if ell <= 128 else 256  # panel width

    def step():
        sk.reset()
        sk.append_csr(indptr, indices, values)
        sk.sketch(out=out)

    for w in range(args.warmup):
        t = time.perf_counter()
        step()
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup}: {time.perf_counter() - t:.3f} s")
    elapsed = float("nan")
    if not args.profile_only:
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(args.steps):
            step()
            log(f"step {k + 1}/{args.steps} done")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    stats = sk.stats()
    value = st_nnz / (elapsed / args.steps)
    log(f"{ms_per_step:.1f} ms/step, {value:.3e} nnz/s, flushes/step={stats['flushes']}")

    # Per-kernel-class pass (after the timed steps): one more step with HIP events around every
    # class's launches on the lane streams, buffers run one lane at a time so that each event
    # pair brackets its kernels alone (concurrent lanes would add other lanes' work to the
    # interval).  The roofline is that of the class with the most device time; its unit is one
    # call of the class (for a sparse product: the main kernel; the long-row fix-up is "fixup").
    roof = None
    phases = {}
    if not args.no_profile:
        sk.set_option(sfd.OPT_LANES, 1)
        sk.set_option(sfd.OPT_PROFILE, 1)
        step()
        torch.cuda.synchronize()
        prof = sk.profile()
        sk.set_option(sfd.OPT_PROFILE, 0)
        sk.set_option(sfd.OPT_LANES, lanes_main)
        for name, p in prof.items():
            if p["calls"]:
                phases[name] = {"ms": p["ms"], "calls": p["calls"], "launches": p["launches"],
                                "avg_call_us": 1e3 * p["ms"] / p["calls"]}
        # the roofline is that of the bandwidth / MFMA classes; the FP64 solvers (Cholesky,
        # eigensolves, shrink factors) are single-workgroup latency-bound kernels, reported apart
        latency_classes = ("chol", "eig", "other")
        dom = max((k for k in prof if k not in latency_classes and prof[k]["calls"]), key=lambda k: prof[k]["ms"])
        p = prof[dom]
        avg_s = p["ms"] / 1e3 / p["calls"]
        if dom in ("gram",):
            achieved = p["flops"] / p["calls"] / avg_s / 1e12
            roof = {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFS, "unit": "TFLOP/s",
                    "frac": achieved / FP32_MFMA_PEAK_TFS, "traffic": None}
        else:
            achieved = p["bytes"] / p["calls"] / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None if (args.csc_bands or args.csc_hot_min) else measured_traffic(dom, args.workload, args.precision)}
        bfk = args.precision == "bf16"
        Lw = 32 if ell <= 32 else 64 if ell <= 64 else 128 if ell <= 128 else 256
        # template arguments <L, U, transposed, BF16 input panel, BF16 output panel, BF16 values,
        # work queue, LDS staging>: the static grid unless the launch was forced or tuned (the
        # BF16 form's bulk of products; its last product, P^T = A'^T Y, writes FP32 from FP32 values)
        b = str(bfk).lower()
        qu = str(args.launch in ("queue", "stage")).lower()
        stg = str(args.launch == "stage").lower()
        tail = ", or a tuned variant" if args.autotune and args.launch == "auto" else ""
        roof["kernel"] = {"spmm_csc": f"k_spmm<{Lw}, {4 if bfk else 8}, true, {b}, {b}, {b}, {qu}, false> "
                                      f"(X = A'^T Y, CSC{tail})",
                          "spmm_csr": f"k_spmm<{Lw}, {4 if bfk else 8}, false, {b}, {b}, {b}, {qu}, {stg}> "
                                      f"(Y = A' X, CSR{tail})"}.get(dom, dom)
        roof["algorithmic_bytes_per_launch"] = p["bytes"] / p["calls"]
        roof["avg_launch_us"] = avg_s * 1e6
        roof["launches"] = p["calls"]
        if dom in ("spmm_csc", "spmm_csr") and stats["flushes"]:
            # what a sparse product actually moves: one panel row (L elements) gathered per stored
            # entry, against the gather rates of 256-byte rows that fit an XCD's L2 (about 20 TB/s)
            # or come from the Infinity Cache (about 8.6 TB/s)
            row_bytes = Lw_main * (2 if args.precision == "bf16" else 4)
            gathered = st_nnz / stats["flushes"] * row_bytes
            roof["gathered_bytes_per_launch"] = gathered
            roof["gathered_TBps"] = gathered / avg_s / 1e12
        roof["timing"] = "HIP events on the lane stream, one-lane pass after the timed steps"
        roof["latency_bound"] = {k: {"ms": prof[k]["ms"], "calls": prof[k]["calls"],
                                     "avg_call_us": 1e3 * prof[k]["ms"] / prof[k]["calls"]}
                                 for k in ("chol", "eig") if prof[k]["calls"]}
        g = prof.get("gram")
        if g and g["calls"]:
            # the panel transform + Gram class on MFMA: achieved FP32 TFLOP/s against the peak and
            # against min(peak, intensity x HBM bandwidth) for its algorithmic bytes
            tf = g["flops"] / (g["ms"] / 1e3) / 1e12
            ai = g["flops"] / max(g["bytes"], 1.0)
            attainable = min(FP32_MFMA_PEAK_TFS, ai * HBM_PEAK_GBS / 1e3)
            roof["gram_mfma"] = {"achieved_tflops": tf, "peak_tflops": FP32_MFMA_PEAK_TFS,
                                 "frac_of_peak": tf / FP32_MFMA_PEAK_TFS, "flop_per_byte": ai,
                                 "attainable_tflops": attainable, "frac_of_attainable": tf / attainable}
        log(f"roofline: {dom} {roof['avg_launch_us']:.1f} us/launch, {achieved:.1f} {roof['unit']}")

    # The forms: fewer steps than the line (each is a whole pass over its workload).
    f_steps = max(1, min(args.steps, args.form_steps))
    f_warmup = max(1, min(args.warmup, 1))
    # The BF16 precision form on the same resident stream: same q, same random blocks; values and
    # panels of SimultaneousIteration in BF16, transforms and Grams on BF16 MFMA.
    forms = {}
    sk_bf = None
    if not args.no_forms and not args.profile_only and args.precision == "fp32":
        sk_bf = sfd.Sketch(st_d, ell, 0.25, 0, precision="bf16", **SKETCH_OPTS)
        out_bf = torch.empty_like(out)

        def step_bf():
            sk_bf.reset()
            sk_bf.append_csr(indptr, indices, values)
            sk_bf.sketch(out=out_bf)

        for _ in range(f_warmup):
            step_bf()
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(f_steps):
            step_bf()
        torch.cuda.synchronize()
        el_bf = time.perf_counter() - t_start
        forms["bf16"] = {"value": st_nnz / (el_bf / f_steps), "unit": "nnz/s",
                         "ms_per_step": 1e3 * el_bf / f_steps, "steps": f_steps,
                         "speedup_vs_fp32": (elapsed / args.steps) / (el_bf / f_steps),
                         "rel_frobenius_vs_fp32": gram_rel_distance(out_bf.cpu().numpy(), out.cpu().numpy())}
        log(f"bf16 form: {forms['bf16']['ms_per_step']:.1f} ms/step, {forms['bf16']['value']:.3e} nnz/s "
            f"({forms['bf16']['speedup_vs_fp32']:.2f}x FP32)")

    # The batched form: the first `batch_streams` streams of the 4,096-stream recipe (d = 2e4,
    # ell = 32, log-uniform lengths 1e3..1e5 rows), resident in HBM, appended in one call and
    # queried; compared with the same streams fed one at a time through a single-stream handle.
    if (not args.no_forms and not args.profile_only and args.precision == "fp32" and args.batch_streams > 0
            and args.workload == "stream1e6"):
        from workloads import batch_stream_d2e4

        t = time.perf_counter()
        bst = [batch_stream_d2e4(s) for s in range(args.batch_streams)]
        bd, bell = bst[0].d, 32
        b_ptr = np.zeros(1 + sum(x.n for x in bst), dtype=np.int64)
        starts = np.zeros(len(bst) + 1, dtype=np.int64)
        pos, base = 1, 0
        for i, x in enumerate(bst):
            b_ptr[pos:pos + x.n] = x.indptr[1:] - x.indptr[0] + base
            pos += x.n
            base += x.nnz
            starts[i + 1] = starts[i] + x.n
        b_nnz = int(base)
        g_ptr = torch.from_numpy(b_ptr).cuda()
        g_idx = torch.from_numpy(np.concatenate([x.indices for x in bst])).cuda()
        g_val = torch.from_numpy(np.concatenate([x.values for x in bst])).cuda()
        log(f"batched form: {len(bst)} streams, {starts[-1]} rows, {b_nnz} nnz generated in "
            f"{time.perf_counter() - t:.1f} s")
        bat = sfd.Batch(len(bst), bd, bell, **BATCH_OPTS)
        b_out = torch.empty((len(bst), bell, bd), dtype=torch.float32, device="cuda")
        sos = np.arange(len(bst), dtype=np.int32)

        def step_batch():
            bat.reset()
            bat.append_csr(sos, starts, g_ptr, g_idx, g_val)
            bat.sketch(out=b_out)

        single = sfd.Sketch(bd, bell, 0.25, 0, **SKETCH_OPTS)
        s_out = torch.empty((bell, bd), dtype=torch.float32, device="cuda")

        def step_single():
            for i in range(len(bst)):
                single.reset()
                single.set_option(sfd.OPT_STREAM_ID, i)
                lo, hi = int(starts[i]), int(starts[i + 1])
                single.append_csr(g_ptr[lo:hi + 1], g_idx, g_val)
                single.sketch(out=s_out)

        res = {}
        for name, fn in (("batched", step_batch), ("single", step_single)):
            for _ in range(f_warmup):
                fn()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(f_steps):
                fn()
            torch.cuda.synchronize()
            res[name] = (time.perf_counter() - t) / f_steps
        forms["batched"] = {"value": b_nnz / res["batched"], "unit": "nnz/s", "ms_per_step": 1e3 * res["batched"],
                            "streams": len(bst), "rows": int(starts[-1]), "nnz": b_nnz, "d": bd, "ell": bell,
                            "single_stream_value": b_nnz / res["single"],
                            "speedup_vs_single_streams": res["single"] / res["batched"],
                            "ratio_vs_fp32_value": (b_nnz / res["batched"]) / value, "steps": f_steps}
        log(f"batched form: {1e3 * res['batched']:.1f} ms/step, {b_nnz / res['batched']:.3e} nnz/s "
            f"({res['single'] / res['batched']:.2f}x one stream at a time)")
        bat.close()
        single.close()
        del g_ptr, g_idx, g_val, b_out

    # The evaluator (sfd_evaluate, FP64 on the GPU): cov-err and proj-err (k = 10) of the timed
    # line's sketch against the whole stream.  Not for the 10^9-entry stream (its 160-step
    # Lanczos runs would take about a minute).
    cov_errs = {}
    if not args.no_forms and not args.profile_only and args.workload in ("stream1e6", "ell200"):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ev = sfd.evaluate(indptr, indices, values, st_d, out, k=10, steps=160)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        forms["eval"] = {"seconds": dt, "cov_err": ev["cov_err"], "proj_err": ev["proj_err"], "k": 10,
                         "cov_max_ritz_residual": ev["cov_max_res"],
                         "lanczos_steps": ev["steps"], "rows": st_n, "nnz": st_nnz, "d": st_d, "ell": ell,
                         "what": "sfd_evaluate of the sketch against the whole stream (two 160-step FP64 "
                                 "Lanczos runs with full reorthogonalisation, CSC build included)"}
        cov_errs["fp32"] = ev["cov_err"]
        log(f"evaluator: cov-err {ev['cov_err']:.4e}, proj-err(k=10) {ev['proj_err']:.4f} of the sketch vs the "
            f"whole stream in {dt:.2f} s")
        if "bf16" in forms:
            evb = sfd.evaluate(indptr, indices, values, st_d, out_bf, k=10, steps=160)
            cov_errs["bf16"] = evb["cov_err"]
            cov_errs["bf16_over_fp32"] = evb["cov_err"] / ev["cov_err"]
            forms["bf16"]["cov_err"] = evb["cov_err"]
            forms["bf16"]["proj_err"] = evb["proj_err"]
            log(f"bf16 form: cov-err {evb['cov_err']:.4e} ({cov_errs['bf16_over_fp32']:.4f}x FP32)")

    # The precision form on its own workloads (ell = 200; d = 1e6, ell = 100) and the batched form
    # on all 4,096 streams, each generated on the device after the 10^6-row stream's handles are
    # released.
    # (measured by child processes before this process started on the GPU, see main's start)
    forms.update(big_forms)

    cpu = None
    parity = None
    eval_check = None
    if args.workload in ("d1e6", "ell200"):
        # The oracle costs a d x ell Householder QR per product (about a second each at d = 1e6,
        # ell = 100), so it checks the device path on the prefix with q = 3 (the same kernels and
        # shapes; the q of the method is only shortened) and is not timed as a baseline.
        t = time.perf_counter()
        Bo, _ = cpu_baseline_prefix(st, ell, 3)
        sk2 = sfd.Sketch(st.d, ell, 0.25, 0, q=3)
        sk2.append_csr(torch.from_numpy(st.indptr).cuda(), torch.from_numpy(st.indices).cuda(),
                       torch.from_numpy(st.values).cuda())
        parity = gram_rel_distance(sk2.sketch().cpu().numpy(), Bo)
        log(f"prefix parity ({st.n} rows, q=3) vs oracle: {parity:.2e} in {time.perf_counter() - t:.1f} s")
        cpu = None
    elif not args.no_cpu_baseline:
        t = time.perf_counter()
        sub, B_oracle, cpu = cpu_baseline(st, ell, min(args.cpu_sample_rows, st.n))
        log(f"cpu baseline: {cpu['value']:.3e} nnz/s in {time.perf_counter() - t:.1f} s")
        # the GPU on the same sample, compared with the oracle (relative Frobenius of B^T B)
        sk2 = sfd.Sketch(st.d, ell, 0.25, 0)
        sk2.append_csr(torch.from_numpy(sub.indptr).cuda(), torch.from_numpy(sub.indices).cuda(),
                       torch.from_numpy(sub.values).cuda())
        Bg = sk2.sketch().cpu().numpy().astype(np.float64)
        parity = gram_rel_distance(Bg, B_oracle)
        log(f"sample parity (rel. Frobenius of B^T B vs oracle): {parity:.2e}")
        # the evaluator on the same sample against scipy's ARPACK on the evaluator's definitions
        # (the sketch's residual A^T A - B^T B is positive semidefinite, so cov-err is its largest
        # eigenvalue over ||A||_F^2)
        if not args.no_forms:
            import scipy.sparse as sps
            import scipy.sparse.linalg as spla

            A_s = sps.csr_matrix((sub.values.astype(np.float64), sub.indices, sub.indptr - sub.indptr[0]),
                                 shape=(sub.n, st.d))
            ev_s = sfd.evaluate(torch.from_numpy(sub.indptr).cuda(), torch.from_numpy(sub.indices).cuda(),
                                torch.from_numpy(sub.values).cuda(), st.d,
                                torch.from_numpy(Bg.astype(np.float32)).cuda(), k=10, steps=160)
            op = spla.LinearOperator((st.d, st.d), dtype=np.float64,
                                     matvec=lambda x: A_s.T @ (A_s @ np.ravel(x)) - Bg.T @ (Bg @ np.ravel(x)))
            lmax = spla.eigsh(op, k=1, which="LA", tol=1e-10, return_eigenvectors=False)[0]
            fro2_ref, proj_ref = cpu_baseline_eval_refs(sub, Bg, 10)
            eval_check = {"cov_err_gpu": ev_s["cov_err"], "cov_err_arpack": float(lmax / fro2_ref),
                          "proj_err_gpu": ev_s["proj_err"], "proj_err_ref": proj_ref,
                          "sample": f"first {sub.n} rows, the GPU sketch of them (ell={ell}), k=10"}
            # cov-err of each form's sketch of the sample against the FP64 oracle's sketch of it, all
            # measured by the FP64 evaluator on the same rows
            g_sub = [torch.from_numpy(a).cuda() for a in (sub.indptr, sub.indices, sub.values)]
            sk3 = sfd.Sketch(st.d, ell, 0.25, 0, precision="bf16")
            sk3.append_csr(*g_sub)
            Bb = sk3.sketch()
            sample_err = {"oracle_fp64": sfd.evaluate(*g_sub, st.d, torch.from_numpy(B_oracle.astype(np.float32)).cuda(),
                                                      steps=160)["cov_err"],
                          "fp32": ev_s["cov_err"],
                          "bf16": sfd.evaluate(*g_sub, st.d, Bb, steps=160)["cov_err"]}
            sample_err["fp32_over_oracle"] = sample_err["fp32"] / sample_err["oracle_fp64"]
            sample_err["bf16_over_oracle"] = sample_err["bf16"] / sample_err["oracle_fp64"]
            sample_err["rows"] = sub.n
            cov_errs["sample"] = sample_err
            log(f"sample cov-err: oracle {sample_err['oracle_fp64']:.6e}, fp32 {sample_err['fp32']:.6e}, "
                f"bf16 {sample_err['bf16']:.6e}")
            log(f"evaluator on the sample: cov-err {ev_s['cov_err']:.6e} (ARPACK {eval_check['cov_err_arpack']:.6e}), "
                f"proj-err {ev_s['proj_err']:.6f} (reference {eval_check['proj_err_ref']:.6f})")
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16 panels, f32 accumulate",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "nnz": st_nnz,
            "ell": ell,
            "buffers_per_step": stats["flushes"],
            "q_last": stats["last_q"],
            "attempts_per_step": stats["attempts"],
            "vs_rejects_per_step": stats["vs_rejects"],
            "lanes": lanes_main,
            "parallelism": "1 GPU",
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "sample_parity_rel_frobenius": parity,
        "cov_err": cov_errs or None,
        "evaluator_check": eval_check,
        "forms": forms,
        "phases": phases,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
