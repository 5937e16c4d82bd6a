"""Benchmark: auto-tuned CSR SpMV on one MI355X.

Workload: the unsymmetric power-law matrix of n = 2,000,000 rows (row
lengths lognormal(2.5, 1) clipped to [1, 5000], uniform distinct columns plus
the diagonal, N(0,1) values, dominant diagonal; about 40.2M entries), FP64
values, x ~ U(-1, 1).  Synthetic, seeded.

A step is one SpMV y = A x with the implementation the run-time selector
(TIME policy: every valid class timed, fastest kept) picked for this matrix.
`value` is the algorithmic HBM rate of those steps: bytes-per-nonzero
accounting (12 B per entry, 4 B per row pointer, 8 B per x and y entry),
divided by the timed wall time of the K steps.

Extra fields on the same JSON line: the FP32-value SpMV rate, the
time-to-1e-10 of GMRES(30) in FP64 and in mixed precision with FP64
refinement (median of 3), the same pair plus the symmetric SpMV rates on the
128^3 27-point stencil stored as its lower triangle, the batched SpMV and
BiCGStab over 512 uneven systems, the trans4-shaped segment-length sweep,
the selector's choices (TIME and LEARNED) and timings, the roofline of the
dominant kernel and the CPU oracle leg.  The oracle leg runs in a thread
pinned to one host core beside the GPU legs: the oracle's SpMV rate (the
baseline), its GMRES(30) time to 1e-10 on both matrices, and the error of
the GPU's FP64 and FP32-value products stated per result (max over rows of
abs(dy) / sum abs(a x)) on both matrices, in both accumulations.

Hardware-counter traffic: before the timed region the script runs a plain
streaming copy of known size (torch.neg over 256 MiB, read once, written
once).  Two rocprofv3 counter runs of this script, one for FETCH_SIZE and one
for WRITE_SIZE, are reduced by `--pmc-summary` into a JSON summary under
profiles/: per SpMV kernel the counter per dispatch, scaled by
known bytes / counter reading of the copy kernel.  The bench reports that
figure as roofline.traffic while the SpMV sources still hash to the value
recorded with the counters, else null.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --pmc-summary FETCH_DIR WRITE_DIR --out FILE
"""
import argparse
import collections
import csv
import glob
import hashlib
import itertools
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CAL_BYTES = 256 << 20
PROFILES = os.path.join(ROOT, "profiles")
# sources whose change invalidates recorded counter figures of an implementation's kernels
COMMON_SOURCES = ("internal.h", "segchunk.h", "spmv_launch.h", "spmv.hip", "plan.hip")
VARIANT_SOURCES = {
    "ROW": ("spmv_row.hip",), "SYM_ATOMIC": ("spmv_row.hip",),
    "NNZ": ("spmv_seg.hip",), "BSS": ("spmv_seg.hip",), "SYM_S3": ("spmv_seg.hip", "sym_layout.h"),
    "XCB": ("spmv_xcb.hip",),
}
# kernels one SpMV of each implementation launches
VARIANT_KERNELS = {
    "ROW": ("k_spmv_row",),
    "NNZ": ("k_spmv_nnz",),
    "BSS": ("k_spmv_bss", "k_bss_fixup"),
    "XCB": ("k_spmv_xcb", "k_xcb_fixup", "k_xcb_combine"),
    "SYM_S3": ("k_spmv_sym_sliced", "k_spmv_sym_s3", "k_sym_block_reduce"),
    "SYM_ATOMIC": ("k_zero", "k_spmv_sym_atomic"),
}


def alg_bytes(n, nnz, val_bytes, x_bytes, y_bytes, idx_bytes=4):
    """Bytes-per-nonzero accounting: every stored entry (value + column index)
    once, the row pointer array once, x once, y once."""
    return nnz * (val_bytes + idx_bytes) + 4 * (n + 1) + x_bytes * n + y_bytes * n


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def spmv_source_hash(variant):
    h = hashlib.sha256()
    for f in COMMON_SOURCES + VARIANT_SOURCES[variant]:
        with open(os.path.join(ROOT, "paper_2405_01599_amd", "csrc", f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def traffic_file(variant, n):
    return os.path.join(PROFILES, f"spmv_{variant.lower()}_fp64_powerlaw_n{n}_traffic.json")


def calibration_copy(torch):
    """The plain streaming copy the counter runs are scaled by."""
    a = torch.full((CAL_BYTES // 8,), 1.0, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()


def stream_rates(torch):
    """Achievable streaming rates on this GPU (HIP events, 10 launches each):
    a 256 MiB read + 256 MiB write elementwise copy, and a 1 GiB read-only
    reduction."""
    a = torch.full((CAL_BYTES // 8,), 1.0, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    big = torch.ones((1 << 30) // 8, dtype=torch.float64, device="cuda")
    out = {}
    for name, fn, by in (("copy_gbs", lambda: torch.neg(a, out=b), 2 * CAL_BYTES),
                         ("read_gbs", lambda: big.sum(), 1 << 30)):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(by / (e0.elapsed_time(e1) / 10 * 1e-3) / 1e9, 1)
    del a, b, big
    return out


def cold_spmv_us(ctx, torch, plan, x, y, reps=5):
    """Single SpMVs after writing a 1 GiB buffer (x, y and the matrix are
    evicted from L2 and the 256 MB MALL first); median of `reps`."""
    flush = torch.empty((1 << 30) // 8, dtype=torch.float64, device="cuda")
    ts = []
    for _ in range(reps):
        flush.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.spmv(plan, x, y)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3)
    del flush
    return round(sorted(ts)[len(ts) // 2], 2)


def _counter_csv(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if len(files) != 1:
        raise SystemExit(f"expected one counter_collection.csv under {d}, found {files}")
    per = collections.defaultdict(list)
    with open(files[0]) as fh:
        for r in csv.DictReader(fh):
            per[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    return per


def _pick_instance(names, frag, precision, instance):
    """The one instantiation of kernel `frag` asked for: FP64 (no float
    template argument) or FP32 (a float argument where one exists, else the
    shared instance), narrowed by the substring `instance` when given."""
    cand = [k for k in names if f"::{frag}<" in k or f"::{frag}(" in k]
    if instance:
        narrowed = [k for k in cand if instance in k]
        cand = narrowed or cand
    if precision == "f32":
        c32 = [k for k in cand if "float" in k]
        cand = c32 or cand
    else:
        cand = [k for k in cand if "float" not in k]
    if len(cand) != 1:
        raise SystemExit(f"kernel {frag}: {len(cand)} {precision} instances found: {[c[:100] for c in cand]}")
    return cand[0]


def pmc_summary(fetch_dir, write_dir, out, variant, n, cmd_fetch, cmd_write, kernels=None, precision="f64",
                instance="", workload=""):
    """Reduce the two counter runs to bytes per launch group (by default one
    FP64 SpMV of `variant`)."""
    F, W = _counter_csv(fetch_dir), _counter_csv(write_dir)
    def mean(per, name, ctr):
        v = per.get((name, ctr))
        if not v:
            raise SystemExit(f"no {ctr} reading for {name[:120]}")
        return sum(v) / len(v), len(v)
    # kernels read in both runs
    names = sorted({k for k, _ in F} & {k for k, _ in W})
    cal = [k for k in names if "neg" in k.lower() and "elementwise" in k.lower()]
    if len(cal) != 1:
        raise SystemExit(f"calibration kernel not found once: {cal}")
    cf, _ = mean(F, cal[0], "FETCH_SIZE")
    cw, _ = mean(W, cal[0], "WRITE_SIZE")
    ff, fw = CAL_BYTES / (cf * 1024.0), CAL_BYTES / (cw * 1024.0)
    ker = {}
    rd = wr = 0.0
    for frag in kernels or VARIANT_KERNELS[variant]:
        name = _pick_instance(names, frag, precision, instance)
        f, nf = mean(F, name, "FETCH_SIZE")
        w, nw = mean(W, name, "WRITE_SIZE")
        ker[frag] = {"name": name[:160], "fetch_kib_per_dispatch": f, "write_kib_per_dispatch": w,
                     "dispatches": [nf, nw], "read_bytes": f * 1024 * ff, "write_bytes": w * 1024 * fw}
        rd += f * 1024 * ff
        wr += w * 1024 * fw
    rep = {"workload": workload or f"power-law CSR n={n}, FP64 SpMV", "variant": variant, "precision": precision,
           "command_fetch": cmd_fetch, "command_write": cmd_write,
           "calibration": {"kernel": cal[0][:160], "bytes_read": CAL_BYTES, "bytes_written": CAL_BYTES,
                           "fetch_kib": cf, "write_kib": cw, "fetch_factor": ff, "write_factor": fw},
           "kernels": ker, "traffic_bytes_per_spmv": {"read": rd, "write": wr, "total": rd + wr},
           "source_sha256": spmv_source_hash(variant) if variant in VARIANT_SOURCES else None}
    with open(out, "w") as fh:
        json.dump(rep, fh, indent=1)
    print(json.dumps(rep["traffic_bytes_per_spmv"]))


def counter_summary(dirs, out, variant, n, nnz, cmds, kernels=None, precision="f64", instance="", workload=""):
    """Reduce counter runs (one directory each) to a markdown table: per
    kernel of one launch group (by default one FP64 SpMV of `variant`),
    each counter's mean per dispatch; with the L2 (TCC) hit and miss
    counts, the hit ratio, and the L2 requests per stored entry."""
    pers = [_counter_csv(d) for d in dirs]
    names = sorted({k for per in pers for k, _ in per})
    title = workload or f"{variant} SpMV (FP64) on the power-law CSR n={n}, nnz={nnz}"
    lines = [f"# {title}: counters per dispatch", "",
             "Commands (repository root, one counter set per run):", "", "```"] + list(cmds) + ["```", ""]
    for frag in kernels or VARIANT_KERNELS[variant]:
        name = _pick_instance(names, frag, precision, instance)
        vals = {}
        for per in pers:
            for (kn, ctr), v in per.items():
                if kn == name:
                    vals[ctr] = sum(v) / len(v)
        lines += [f"## `{frag}`", "", f"`{name[:150]}`", "", "| Counter | Mean per dispatch |", "|---|---|"]
        lines += [f"| {c} | {v:,.0f} |" for c, v in sorted(vals.items())]
        hit, miss = vals.get("TCC_HIT_sum"), vals.get("TCC_MISS_sum")
        if hit is not None and miss is not None and hit + miss > 0:
            lines += [f"| L2 hit ratio (TCC_HIT / (TCC_HIT + TCC_MISS)) | {hit / (hit + miss):.4f} |"]
        if "TCC_REQ_sum" in vals:
            lines += [f"| L2 requests per stored entry | {vals['TCC_REQ_sum'] / nnz:.3f} |"]
        lines.append("")
    with open(out, "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


def recorded_traffic(variant, n):
    """HBM bytes per SpMV from the committed counter summary, if it still
    describes the current kernels; (value, note)."""
    path = traffic_file(variant, n)
    if not os.path.exists(path):
        return None, "no counter summary for this kernel and workload"
    with open(path) as fh:
        rep = json.load(fh)
    if rep.get("source_sha256") != spmv_source_hash(variant):
        return None, "SpMV sources changed since the counters were taken"
    return round(rep["traffic_bytes_per_spmv"]["total"]), os.path.relpath(path, ROOT)


def host_cpu_info():
    """The host CPU as /proc/cpuinfo and sysfs describe it."""
    info = {"model_name": "unknown"}
    try:
        with open("/proc/cpuinfo") as fh:
            first = fh.read().split("\n\n")[0]
        for ln in first.splitlines():
            k, _, v = ln.partition(":")
            k, v = k.strip(), v.strip()
            if k == "model name":
                info["model_name"] = v
            elif k in ("cpu family", "model", "stepping", "cpu MHz", "cache size"):
                info[k.replace(" ", "_")] = v
    except OSError:
        pass
    try:
        with open("/sys/devices/system/cpu/cpu0/cpufreq/cpuinfo_max_freq") as fh:
            info["max_mhz"] = round(int(fh.read().strip()) / 1000)
    except (OSError, ValueError):
        pass
    info["nproc"] = os.cpu_count()
    try:
        info["usable_cores"] = len(os.sched_getaffinity(0))
    except OSError:
        pass
    return info


class OracleLeg:
    """The CPU oracle's part of the run, in a thread of its own that runs
    beside the GPU legs (the oracle's C calls release the interpreter lock),
    pinned to one host core:
      - the baseline: full serial FP64 SpMVs of the power-law matrix for
        about budget_s;
      - the oracle's GMRES(30) + Jacobi to 1e-10 (MGS, b = 1) on the
        power-law matrix and on the 27-point stencil 128^3 (full storage);
      - the per-result error of the GPU's products handed over by check():
        max over rows of abs(y - y_oracle) / sum abs(a x), against the
        oracle on the FP64 inputs and on the FP32-rounded inputs."""

    def __init__(self, A, x, budget_s=10.0, gmres=True):
        import queue
        import threading
        self.A, self.x, self.budget_s, self.gmres = A, x, budget_s, gmres
        self.result, self.error, self.errors = None, None, {}
        self.q = queue.Queue()
        self.thread = threading.Thread(target=self._run, daemon=True)
        self.thread.start()

    def check(self, name, A, x64, ys):
        """Queue the GPU results ys = {label: (y, inputs)} of A x for
        comparison; inputs is "f64" or "f32" (values and x rounded)."""
        self.q.put((name, A, x64, ys))

    def _run(self):
        try:
            self.result = self._measure()
            while True:
                item = self.q.get()
                if item is None:
                    break
                self._compare(*item)
        except Exception as e:  # reported, not fatal to the GPU legs
            self.error = repr(e)

    def _compare(self, name, A, x64, ys):
        import gen
        import oracle
        ref = {"f64": oracle.spmv(A, x64)}
        if any(inp == "f32" for _, inp in ys.values()):
            A32 = gen.CSR(A.n, A.ncols, A.rowptr, A.colind, A.val.astype(np.float32).astype(np.float64),
                          sym_lower=A.sym_lower)
            ref["f32"] = oracle.spmv(A32, x64.astype(np.float32).astype(np.float64))
        res = {}
        for label, (y, inp) in ys.items():
            yo, so = ref["f64"]
            e = fp32_error_per_result(y, yo, so)
            if inp == "f32":
                yr, sr = ref["f32"]
                e["vs_rounded_inputs"] = fp32_error_per_result(y, yr, sr)["max_abs_dy_over_s"]
            res[label] = e
        self.errors[name] = res

    def _measure(self):
        import gen
        import oracle
        host = host_cpu_info()
        core = max(os.sched_getaffinity(0))
        os.sched_setaffinity(0, {core})  # this thread only
        A, x = self.A, self.x
        reps = 0
        t0 = time.perf_counter()
        while True:
            oracle.spmv(A, x)
            reps += 1
            el = time.perf_counter() - t0
            if el >= self.budget_s:
                break
        by = alg_bytes(A.n, A.nnz, 8, 8, 8)
        out = {"value": round(by * reps / el / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"{reps} full FP64 SpMVs of the n={A.n} power-law matrix ({el:.1f} s, 1 thread)",
               "pinned_core": core, "host": host}
        if self.gmres:
            for name, M in (("gmres_powerlaw", A), ("gmres_sym27", None)):
                if M is None:
                    L = gen.stencil27(128, lower=True)
                    rp, ci, v = oracle.sym_expand(L)
                    M = gen.CSR(L.n, L.n, rp, ci, v)
                t0 = time.perf_counter()
                r = oracle.gmres(M, np.ones(M.n), m=30, tol=1e-10, precond=1)
                out[name] = {"s": round(time.perf_counter() - t0, 3), "iters": r["iters"], "cycles": r["cycles"],
                             "relres": r["relres"], "status": r["status"],
                             "what": "oracle GMRES(30), MGS, right Jacobi, b = 1, x0 = 0, to 1e-10, 1 core"}
        return out

    def join(self):
        self.q.put(None)
        self.thread.join()
        if self.error:
            return {"error": self.error}, self.errors
        return self.result, self.errors


def fp32_error_per_result(y, yo, s):
    """max over rows of abs(y - yo) / s, and whether the rows with s = 0
    are exactly 0."""
    nz = s > 0
    return {"max_abs_dy_over_s": float(np.max(np.abs(y[nz] - yo[nz]) / s[nz])) if nz.any() else 0.0,
            "zero_rows_exact": bool(np.all(y[~nz] == 0))}


def gmres_pair(ctx, xab, torch, plan, n, reps=3):
    """Time-to-1e-10 of GMRES(30) with Jacobi, FP64 and mixed precision
    (FP32 inner solve to the default inner tolerance 1e-6, FP64
    refinement): b = 1, x0 = 0, median of `reps`.  Also the mixed-precision
    solve with looser inner tolerances (more refinements, fewer inner
    steps each)."""
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    res = {}

    def run(mode, **kw):
        runs = []
        for _ in range(reps):
            xs, inf, st = ctx.gmres(plan, b, m=30, tol=1e-10, mode=mode, precond=xab.PRECOND_JACOBI, **kw)
            runs.append(inf)
        runs.sort(key=lambda r: r["seconds"])
        med = runs[len(runs) // 2]
        return {"s": round(med["seconds"], 5), "iters": med["iters"], "restarts": med["restarts"],
                "refinements": med["refinements"], "relres": med["true_relres"], "status": med["status"]}

    res["fp64"] = run(xab.MODE_FP64)
    res["ir"] = run(xab.MODE_IR)
    res["ir_speedup"] = round(res["fp64"]["s"] / res["ir"]["s"], 3)
    res["ir_inner_tol"] = {}
    for it in (1e-3, 1e-4):
        r = run(xab.MODE_IR, inner_tol=it)
        r["speedup_vs_fp64"] = round(res["fp64"]["s"] / r["s"], 3)
        res["ir_inner_tol"][f"{it:g}"] = r
    return res


def ortho_menu_leg(ctx, xab, torch, plan, n):
    """FP64 GMRES(30) with Jacobi to 1e-10 under each orthogonalisation and
    the accuracy policy; median of 3 each."""
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    res = {}
    for name, o in (("dgks", xab.ORTHO_DGKS), ("cgs", xab.ORTHO_CGS), ("mgs", xab.ORTHO_MGS),
                    ("bcgs", xab.ORTHO_BCGS), ("policy", xab.ORTHO_POLICY)):
        runs = sorted((ctx.gmres(plan, b, m=30, tol=1e-10, precond=xab.PRECOND_JACOBI, ortho=o)[1] for _ in range(3)),
                      key=lambda r: r["seconds"])
        med = runs[1]
        res[name] = {"s": round(med["seconds"], 5), "iters": med["iters"], "relres": med["true_relres"],
                     "status": med["status"], "faults": med["faults"]}
    # mixed precision under the policy: the inner solve's requirement (1e-6) selects BCGS
    runs = sorted((ctx.gmres(plan, b, m=30, tol=1e-10, mode=xab.MODE_IR, precond=xab.PRECOND_JACOBI,
                             ortho=xab.ORTHO_POLICY)[1] for _ in range(3)), key=lambda r: r["seconds"])
    med = runs[1]
    res["ir_policy"] = {"s": round(med["seconds"], 5), "iters": med["iters"], "relres": med["true_relres"],
                        "status": med["status"], "ortho": med["ortho"]}
    return res


def restart_tuning_leg(ctx, xab, torch, plan, n):
    """Restart-length tuning by the MM ratio: FP64 GMRES with Jacobi from
    m = 5, fixed vs grown by 5 (up to 30) after each cycle whose MM ratio is
    below 10; median of 3 each."""
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    res = {}
    for name, kw in (("fixed_m5", {}), ("tuned_m5_step5_max30", dict(restart_step=5, m_max=30, mm_ratio=10.0))):
        runs = sorted((ctx.gmres(plan, b, m=5, tol=1e-10, precond=xab.PRECOND_JACOBI, **kw)[1] for _ in range(3)),
                      key=lambda r: r["seconds"])
        med = runs[1]
        res[name] = {"s": round(med["seconds"], 5), "iters": med["iters"], "cycles": med["restarts"],
                     "m_final": med["m_final"], "relres": med["true_relres"], "status": med["status"]}
    return res


def lanczos_leg(ctx, xab, torch, gen, plan, g):
    """Thick-restart Lanczos on the 27-point stencil (section 4.3 setting: 10
    eigenpairs to 1e-8), both ends of the spectrum: a fixed basis of 30
    vectors, and restart-length tuning from 20 (m += 5 up to 60 when the MM
    ratio of 5 per-cycle samples is below 2); wall time of the call and the
    distance of every eigenvalue to the stencil's closed-form spectrum."""
    import numpy as np
    t = 1.0 + 2.0 * np.cos(np.arange(1, g + 1) * np.pi / (g + 1))
    lam = np.sort((28.0 - np.einsum("i,j,k->ijk", t, t, t)).ravel())
    v0 = torch.from_numpy(gen.uniform_vec(g ** 3, 5)).cuda()
    out = {}
    runs = (("fixed_m30", dict(m=30)),
            ("tuned_m20_to_60", dict(m=20, restart_step=5, m_max=60, mm_ratio=2.0, window=5)))
    ends = ((xab.EIG_LARGEST, "largest"), (xab.EIG_SMALLEST, "smallest"))
    for (which, name), (tag, kw) in itertools.product(ends, runs):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, X, info, st = ctx.lanczos(plan, v0, nev=10, tol=1e-8, which=which, max_time_s=60.0, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        err = max(float(np.min(np.abs(lam - v))) for v in ev) / info["anrm"]
        out[f"{name}_{tag}"] = {
            "s": round(wall, 4), "status": st, "matvecs": info["iters"], "restarts": info["restarts"],
            "m_final": info["m_final"], "ms_per_matvec": round(wall / max(1, info["iters"]) * 1e3, 4),
            "max_resid_rel": info["max_resid"], "closed_form_err_rel": err,
            "evals": [round(float(v), 12) for v in (ev[0], ev[-1])]}
        del X
    return out


def arnoldi_leg(ctx, xab, torch, gen, plan_c2, n_c2):
    """Implicitly restarted Arnoldi (10 eigenvalues to 1e-8): the power-law
    matrix's largest-magnitude ones (fixed m = 30), and the 128^3
    convection-diffusion operator's largest-real-part ones, fixed m = 30
    against restart-length tuning from 20 (m += 5 up to 60 when the MM
    ratio of 5 per-cycle samples is below 2), with the distance of every
    value to that operator's closed-form spectrum."""
    import numpy as np
    out = {}
    v0 = torch.from_numpy(gen.uniform_vec(n_c2, 5)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, X, info, st = ctx.arnoldi(plan_c2, v0, nev=10, m=30, tol=1e-8, which=xab.EIG_MAGNITUDE, max_time_s=60.0)
    torch.cuda.synchronize()
    out["powerlaw_largest_magnitude_m30"] = {
        "s": round(time.perf_counter() - t0, 4), "status": st, "matvecs": info["iters"],
        "restarts": info["restarts"], "max_resid_rel": info["max_resid"],
        "evals": [str(complex(round(v.real, 9), round(v.imag, 9))) for v in (ev[0], ev[-1])]}
    del X
    g, beta = 128, 0.02
    A = gen.convdiff3d(g, beta)
    k = np.arange(1, g + 1)
    lx = 2.0 + 2.0 * np.sqrt(1.0 - beta * beta) * np.cos(k * np.pi / (g + 1))
    ly = 2.0 - 2.0 * np.cos(k * np.pi / (g + 1))
    lam = np.sort((lx[:, None, None] + ly[None, :, None] + ly[None, None, :]).ravel())
    M = ctx.matrix_from_csr(A)
    plan, sinfo = ctx.select(M, xab.TIME)
    v0 = torch.from_numpy(gen.uniform_vec(A.n, 5)).cuda()
    out["convdiff_workload"] = f"7-point convection-diffusion {g}^3, beta = {beta}: n={A.n} nnz={A.nnz}"
    out["convdiff_selected"] = plan.describe()["variant"]
    for tag, kw in (("fixed_m30", dict(m=30)),
                    ("tuned_m20_to_60", dict(m=20, restart_step=5, m_max=60, mm_ratio=2.0, window=5))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, X, info, st = ctx.arnoldi(plan, v0, nev=10, tol=1e-8, which=xab.EIG_LARGEST, max_time_s=60.0, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[f"convdiff_largest_real_{tag}"] = {
            "s": round(wall, 4), "status": st, "matvecs": info["iters"], "restarts": info["restarts"],
            "m_final": info["m_final"], "ms_per_matvec": round(wall / max(1, info["iters"]) * 1e3, 4),
            "max_resid_rel": info["max_resid"],
            "closed_form_err_rel": max(float(np.min(np.abs(lam - v.real))) for v in ev) / info["anrm"],
            "max_abs_imag": float(np.max(np.abs(ev.imag)))}
        del X
    plan.close()
    M.close()
    return out


def _csr_from_coo(gen, rows, cols, vals, nr, nc, lower=False, name=""):
    """CSR from entries already ordered by (row, column)."""
    import numpy as np
    rp = np.zeros(nr + 1, dtype=np.int32)
    rp[1:] = np.cumsum(np.bincount(rows, minlength=nr))
    return gen.CSR(nr, nc, rp, np.ascontiguousarray(cols, dtype=np.int32), np.ascontiguousarray(vals),
                   sym_lower=lower, name=name)


def _time_selected(ctx, xab, torch, gen, S, seed):
    """TIME-select an implementation for S and time its FP64 SpMV (HIP
    events, 100 launches); returns (us, class, variant)."""
    M = ctx.matrix_from_csr(S)
    plan, info = ctx.select(M, xab.TIME)
    x = torch.from_numpy(gen.uniform_vec(S.ncols, seed)).cuda()
    y = torch.empty(S.n, dtype=torch.float64, device="cuda")
    ms = ctx.time_spmv(plan, x, y, warmup=5, reps=100)
    out = (round(ms * 1e3, 2), int(info.chosen), plan.describe()["variant"])
    plan.close()
    M.close()
    return out


def shard_leg(ctx, xab, torch, gen, A):
    """One GPU's share of an 8-GPU row decomposition, at its real shape.
    Power-law: rows [0, n/8) against the whole x (what each GPU multiplies
    after the all-gather of x).  27-point 128^3, lower storage, 16 planes
    [56, 72): the diagonal block (symmetric, lower) plus the coupling block
    C to the previous shard's last 16,513 rows and its transpose (the
    partial y sent back), each with its own TIME-selected implementation."""
    import numpy as np
    out = {}
    ns = A.n // 8
    nz = int(A.rowptr[ns])
    S = gen.CSR(ns, A.ncols, A.rowptr[:ns + 1].copy(), A.colind[:nz], A.val[:nz], name="powerlaw_shard")
    us, k, var = _time_selected(ctx, xab, torch, gen, S, 12)
    by = 12 * nz + 4 * (ns + 1) + 8 * A.ncols + 8 * ns
    out["powerlaw_rows_div8"] = {"rows": ns, "nnz": nz, "us": us, "class": k, "variant": var,
                                 "gbs": round(by / (us * 1e-6) / 1e9, 1),
                                 "allgather_bytes_per_gpu": 8 * (A.ncols - ns)}
    g = 128
    L = gen.stencil27(g, lower=True)
    r0, r1, H = 56 * g * g, 72 * g * g, g * g + g + 1
    n_s = r1 - r0
    z0, z1 = int(L.rowptr[r0]), int(L.rowptr[r1])
    rows = np.repeat(np.arange(n_s), np.diff(L.rowptr[r0:r1 + 1]))
    cols, vals = L.colind[z0:z1].astype(np.int64), L.val[z0:z1]
    own = cols >= r0
    D = _csr_from_coo(gen, rows[own], cols[own] - r0, vals[own], n_s, n_s, lower=True, name="st27_shard_diag")
    C = _csr_from_coo(gen, rows[~own], cols[~own] - (r0 - H), vals[~own], n_s, H, name="st27_shard_coupling")
    order = np.lexsort((rows[~own], cols[~own]))
    CT = _csr_from_coo(gen, (cols[~own] - (r0 - H))[order], rows[~own][order], vals[~own][order], H, n_s,
                       name="st27_shard_coupling_T")
    parts, tot_us, tot_by = {}, 0.0, 0
    for name, S, by in (("diag_sym", D, 12 * D.nnz + 4 * (n_s + 1) + 16 * n_s),
                        ("coupling", C, 12 * C.nnz + 4 * (n_s + 1) + 8 * H + 8 * n_s),
                        ("coupling_T", CT, 12 * CT.nnz + 4 * (H + 1) + 8 * n_s + 8 * H)):
        us, k, var = _time_selected(ctx, xab, torch, gen, S, 13)
        parts[name] = {"rows": S.n, "cols": S.ncols, "nnz": S.nnz, "us": us, "class": k, "variant": var}
        tot_us += us
        tot_by += by
    out["st27_planes_16"] = {"rows": n_s, "halo_rows": H, "halo_bytes_per_side": 8 * H, **parts,
                             "us_total": round(tot_us, 2), "gbs": round(tot_by / (tot_us * 1e-6) / 1e9, 1)}
    return out


def sym_stencil_leg(ctx, xab, torch, gen, gmres=True, eig=True, oracle_leg=None):
    """Symmetric SpMV from lower storage on the 128^3 27-point stencil:
    TIME-selected implementation, FP64 and FP32 values (FP64 accumulation),
    then GMRES(30) FP64 vs mixed precision on it, and the Lanczos leg."""
    L = gen.stencil27(128, lower=True)
    M = ctx.matrix_from_csr(L, with_f32=True)
    plan, info = ctx.select(M, xab.TIME)
    x = torch.from_numpy(gen.uniform_vec(L.n, 13)).cuda()
    y = torch.empty(L.n, dtype=torch.float64, device="cuda")
    ms64 = ctx.time_spmv(plan, x, y, warmup=5, reps=100)
    cold64 = cold_spmv_us(ctx, torch, plan, x, y)
    x32, y32 = x.float(), y.float()
    ms32 = ctx.time_spmv(plan, x32, y32, acc=xab.F64, warmup=5, reps=100)
    if oracle_leg:
        xh = x.cpu().numpy()
        ys = {"fp64": (ctx.spmv(plan, x).cpu().numpy(), "f64"),
              "fp32_values_acc_fp64": (ctx.spmv(plan, x32, ydtype=torch.float32, acc=xab.F64).double().cpu().numpy(),
                                       "f32"),
              "fp32_values_acc_fp32": (ctx.spmv(plan, x32, ydtype=torch.float32, acc=xab.F32).double().cpu().numpy(),
                                       "f32")}
        oracle_leg.check("sym27", L, xh, ys)
    by64, by32 = alg_bytes(L.n, L.nnz, 8, 8, 8), alg_bytes(L.n, L.nnz, 4, 4, 4)
    out = {"workload": f"27-point stencil 128^3, lower triangle stored: n={L.n} nnz_L={L.nnz}",
           "selected": plan.describe(), "chosen_class": int(info.chosen),
           "us_per_class": {k: round(float(info.time_ms[k]) * 1e3, 2) for k in range(xab.NCLASSES) if info.valid[k]},
           "fp64": {"us": round(ms64 * 1e3, 2), "cold_us": cold64, "gbs": round(by64 / (ms64 * 1e-3) / 1e9, 1),
                    "frac": round(by64 / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "gflops": round(2 * (2 * L.nnz - L.n) / (ms64 * 1e-3) / 1e9, 1)},
           "fp32_values": {"us": round(ms32 * 1e3, 2), "gbs": round(by32 / (ms32 * 1e-3) / 1e9, 1),
                           "frac": round(by32 / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}
    if gmres:
        out["gmres"] = gmres_pair(ctx, xab, torch, plan, L.n)
        out["gmres_restart_tuning"] = restart_tuning_leg(ctx, xab, torch, plan, L.n)
    if eig:
        out["lanczos"] = lanczos_leg(ctx, xab, torch, gen, plan, 128)
    plan.close()
    M.close()
    return out


def batch_leg(ctx, xab, torch, gen):
    """512 uneven systems (banded and random rows, n log-uniform in
    [1000, 65536]) as one block-diagonal CSR: the persistent batched SpMV in
    FP64 and FP32 (HIP events on the context stream, 50 launches), and
    batched BiCGStab with Jacobi to 1e-10 (FP64) / 1e-5 (FP32), graph-captured
    iterations vs eager launches."""
    B = gen.batch()
    out = {"workload": f"512 systems, n={B.n} nnz={B.nnz}, block-diagonal CSR"}
    for dt, tol, vb in (("f64", 1e-10, 8), ("f32", 1e-5, 4)):
        # the segmented-scan tiles first, for comparison (graph-captured BiCGStab only)
        bt = ctx.batch(B, dtype=dt, tiles=True)
        b = torch.ones(B.n, dtype=bt.dtype, device="cuda")
        ctx.bicgstab(bt, b, tol=tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.bicgstab(bt, b, tol=tol)
        torch.cuda.synchronize()
        tiles_s = round(time.perf_counter() - t0, 5)
        bt.close()
        del b
        bt = ctx.batch(B, dtype=dt)
        x = torch.ones(B.n, dtype=bt.dtype, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            bt.spmv(x, y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(50):
            bt.spmv(x, y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 50
        by = alg_bytes(B.n, B.nnz, vb, vb, vb)
        leg = {"layout": bt.layout, "spmv_us": round(ms * 1e3, 2), "spmv_gbs": round(by / (ms * 1e-3) / 1e9, 1),
               "spmv_frac": round(by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "bicgstab_graph_tiles_s": tiles_s}
        b = torch.ones(B.n, dtype=bt.dtype, device="cuda")
        for graph in (True, False):
            ctx.bicgstab(bt, b, tol=tol, graph=graph)  # warm (graph instantiation, code paths)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xs, per, agg, st = ctx.bicgstab(bt, b, tol=tol, graph=graph)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            leg["bicgstab_graph" if graph else "bicgstab_eager"] = {
                "s": round(wall, 5), "status": st, "max_iters": max(p["iters"] for p in per),
                "converged": sum(1 for p in per if p["status"] == 0),
                "max_relres": max(p["true_relres"] for p in per)}
        out[dt] = leg
        bt.close()
        del x, y, b
    return out


def xcb_gather_reference(ctx, xab, torch, gen, A, ev_ms, j_per_lane):
    """What the random x gathers cost the column-blocked SpMV: the same
    matrix with every column moved into the first 2048 columns of its own
    column block (same rows, lengths, values and blocks, so the same entry
    stream, tiles and partial sums, but each XCD gathers from a 16 KB slice
    of x that stays in its CUs' L1 caches), timed with the same entries per
    lane."""
    k = (A.colind.astype(np.int64) * 8) // A.ncols
    lo = (k * A.ncols) // 8
    ci = (lo + A.colind.astype(np.int64) % 2048).astype(np.int32)
    L = gen.CSR(A.n, A.ncols, A.rowptr, ci, A.val, name="powerlaw_local_columns")
    M = ctx.matrix_from_csr(L)
    P = ctx.plan(M, xab.XCB, j_per_lane=j_per_lane)
    x = torch.from_numpy(gen.uniform_vec(A.n, 12)).cuda()
    y = torch.empty(A.n, dtype=torch.float64, device="cuda")
    ms = ctx.time_spmv(P, x, y, warmup=5, reps=100)
    P.close()
    M.close()
    return {"random_columns_us": round(ev_ms * 1e3, 2), "local_columns_us": round(ms * 1e3, 2),
            "random_gather_share": round(1.0 - ms / ev_ms, 4),
            "gathers_per_s": round(A.nnz / (ev_ms * 1e-3) / 1e9, 1), "unit_gathers": "G/s",
            "what": "same matrix, each column moved into the first 2048 columns of its XCD column block"}


def c1_leg(ctx, xab, torch, gen):
    """The small case: the 64 x 64 Laplacian, general and lower-stored:
    device time per FP64 SpMV (HIP events, 100 launches) of every class
    that applies (launch-latency bound at this size)."""
    out = {}
    for key, lower, classes in (("general", False, xab.GENERAL_CLASSES), ("lower", True, xab.SYM_CLASSES)):
        A = gen.laplacian2d(64, lower=lower)
        M = ctx.matrix_from_csr(A)
        x = torch.from_numpy(gen.uniform_vec(A.n, 1)).cuda()
        y = torch.empty(A.n, dtype=torch.float64, device="cuda")
        us = {}
        for k in classes:
            try:
                P = ctx.plan_class(M, k)
            except xab.XabError:
                continue
            us[k] = round(ctx.time_spmv(P, x, y, warmup=5, reps=100) * 1e3, 2)
            P.close()
        out[key] = {"n": A.n, "nnz": A.nnz, "us_per_class": us}
        M.close()
    return out


def trans4_leg(ctx, xab, torch, gen):
    """The very unbalanced trans4 shape of the paper's segment-length sweep
    (one row of 114,910 entries among 116,835 rows, 749,800 entries):
    device time per FP64 SpMV (HIP events, 100 launches) of the branchless
    segmented scan at J = 1 .. 32 entries per lane against the row-based
    split at 1, 8 and 64 lanes per row and the nnz-based split."""
    A = gen.trans4_like()
    M = ctx.matrix_from_csr(A)
    x = torch.from_numpy(gen.uniform_vec(A.n, 22)).cuda()
    y = torch.empty(A.n, dtype=torch.float64, device="cuda")
    out = {"workload": f"trans4-shaped CSR n={A.n} nnz={A.nnz}, longest row {int(np.diff(A.rowptr).max())}"}

    def t(variant, **kw):
        P = ctx.plan(M, variant, **kw)
        ms = ctx.time_spmv(P, x, y, warmup=5, reps=100)
        P.close()
        return round(ms * 1e3, 2)
    out["bss_us_by_j"] = {j: t(xab.BSS, j_per_lane=j) for j in (1, 2, 4, 8, 16, 32)}
    out["row_us_by_lanes"] = {sl: t(xab.ROW, lanes_per_row=sl) for sl in (1, 8, 64)}
    out["nnz_us_by_tile"] = {tt: t(xab.NNZ, tile_nnz=tt) for tt in (2048, 8192)}
    best_bss = min(out["bss_us_by_j"].values())
    out["bss_best_vs_row1"] = round(out["row_us_by_lanes"][1] / best_bss, 2)
    out["bss_best_vs_best_row"] = round(min(out["row_us_by_lanes"].values()) / best_bss, 2)
    M.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-gmres", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the symmetric 27-point stencil leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-system batch leg")
    ap.add_argument("--no-eig", action="store_true", help="skip the Lanczos and Arnoldi legs")
    ap.add_argument("--no-shard", action="store_true", help="skip the one-GPU-share leg")
    ap.add_argument("--no-c1", action="store_true", help="skip the 64 x 64 Laplacian leg")
    ap.add_argument("--no-gather-ref", action="store_true",
                    help="skip the local-column XCB reference (counter runs: keeps its dispatches out of the means)")
    ap.add_argument("--n", type=int, default=2_000_000)
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--counter-summary", nargs="+", metavar="DIR",
                    help="reduce counter runs (L2 hits, misses, requests) to a markdown table at --out")
    ap.add_argument("--nnz", type=int, default=0, help="stored entries of the workload (--counter-summary)")
    ap.add_argument("--cmds", nargs="*", default=[], help="the counter runs' commands (--counter-summary)")
    ap.add_argument("--variant", default="XCB")
    ap.add_argument("--kernels", nargs="*", default=None, help="kernel names to summarise (default: the variant's)")
    ap.add_argument("--precision", choices=("f64", "f32"), default="f64", help="which instances to summarise")
    ap.add_argument("--instance", default="", help="substring that picks one of several instances")
    ap.add_argument("--workload", default="", help="workload text of the summary")
    ap.add_argument("--out")
    ap.add_argument("--cmd-fetch", default="")
    ap.add_argument("--cmd-write", default="")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, args.out, args.variant, args.n, args.cmd_fetch, args.cmd_write,
                    args.kernels, args.precision, args.instance, args.workload)
        return
    if args.counter_summary:
        counter_summary(args.counter_summary, args.out, args.variant, args.n, args.nnz, args.cmds,
                        args.kernels, args.precision, args.instance, args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding "
              "is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch
    import gen
    import paper_2405_01599_amd as xab

    log("generating the power-law matrix")
    A = gen.powerlaw(args.n, seed=2)
    x64 = gen.uniform_vec(A.n, 12)
    oracle_leg = None if args.no_cpu else OracleLeg(A, x64, gmres=not args.no_gmres)
    ctx = xab.Context(0)
    M = ctx.matrix_from_csr(A, with_f32=True)
    xd = torch.from_numpy(x64).cuda()
    xd32 = xd.float()
    y = torch.empty(A.n, dtype=torch.float64, device="cuda")
    y32 = torch.empty(A.n, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()

    calibration_copy(torch)

    log("selecting (LEARNED, then TIME policy)")
    ctx.select(M, xab.LEARNED)[0].close()  # first call loads the shipped model
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lplan, linfo = ctx.select(M, xab.LEARNED)
    torch.cuda.synchronize()
    learned = {"chosen_class": int(linfo.chosen), "select_ms": round((time.perf_counter() - t0) * 1e3, 2)}
    lplan.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan, info = ctx.select(M, xab.TIME)
    torch.cuda.synchronize()
    time_wall_ms = (time.perf_counter() - t0) * 1e3
    chosen = int(info.chosen)
    times = {k: round(float(info.time_ms[k]) * 1e3, 2) for k in range(xab.NCLASSES) if info.valid[k]}
    plan_mb = {k: round(int(info.bytes[k]) / 1e6, 2) for k in range(xab.NCLASSES) if info.valid[k]}
    # the MEMORY policy: least plan memory, then speed
    mplan, minfo = ctx.select(M, xab.MEMORY)
    memory = {"chosen_class": int(minfo.chosen), "plan_mb": round(mplan.bytes / 1e6, 2),
              "us": round(float(minfo.time_ms[minfo.chosen]) * 1e3, 2)}
    mplan.close()
    torch.cuda.synchronize()

    # timed region: K steps of the selected FP64 SpMV
    for _ in range(args.warmup):
        ctx.spmv(plan, xd, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.spmv(plan, xd, y)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall / args.steps * 1e3
    by64 = alg_bytes(A.n, A.nnz, 8, 8, 8)
    gbs = by64 / (wall / args.steps) / 1e9

    # dominant kernel: device time per launch from HIP events on the
    # context stream (the stream the kernels are queued on)
    ev_ms = ctx.time_spmv(plan, xd, y, warmup=5, reps=100)
    ach = by64 / (ev_ms * 1e-3) / 1e9
    variant = plan.describe()["variant"].upper()
    traffic, tnote = recorded_traffic(variant, A.n)
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_source": tnote,
                "kernel": f"{variant} SpMV: " + " + ".join(VARIANT_KERNELS.get(variant, ())),
                "bytes_per_launch": by64, "us_per_launch": round(ev_ms * 1e3, 2)}

    cold = cold_spmv_us(ctx, torch, plan, xd, y)
    stream = stream_rates(torch)
    gather_ref = None
    if variant == "XCB" and not args.no_gather_ref:
        gather_ref = xcb_gather_reference(ctx, xab, torch, gen, A, ev_ms, plan.describe()["j_per_lane"])

    # FP32 values and x, FP64 accumulation, FP32 y (the inner SpMV of GMRES-IR)
    plan32 = ctx.plan_class(M, chosen)
    ev32 = ctx.time_spmv(plan32, xd32, y32, acc=xab.F64, warmup=5, reps=100)
    by32 = alg_bytes(A.n, A.nnz, 4, 4, 4)
    fp32 = {"gbs": round(by32 / (ev32 * 1e-3) / 1e9, 1), "us": round(ev32 * 1e3, 2),
            "frac": round(by32 / (ev32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "speedup_vs_fp64": round(ev_ms / ev32, 3)}
    if oracle_leg:
        # results handed to the oracle leg for the per-result error
        ys = {"fp64": (ctx.spmv(plan, xd).cpu().numpy(), "f64"),
              "fp32_values_acc_fp64": (ctx.spmv(plan32, xd32, ydtype=torch.float32, acc=xab.F64).double().cpu().numpy(),
                                       "f32"),
              "fp32_values_acc_fp32": (ctx.spmv(plan32, xd32, ydtype=torch.float32, acc=xab.F32).double().cpu().numpy(),
                                       "f32")}
        oracle_leg.check("powerlaw", A, x64, ys)

    gm = None
    if not args.no_gmres:
        log("GMRES(30) FP64 vs mixed precision (power-law)")
        gm = gmres_pair(ctx, xab, torch, plan, A.n)
        gm["ortho_menu"] = ortho_menu_leg(ctx, xab, torch, plan, A.n)

    arn = None
    if not args.no_eig:
        log("Arnoldi (power-law, convection-diffusion)")
        arn = arnoldi_leg(ctx, xab, torch, gen, plan, A.n)

    c3 = None
    if not args.no_c3:
        log("symmetric 27-point stencil 128^3 (lower storage)")
        c3 = sym_stencil_leg(ctx, xab, torch, gen, gmres=not args.no_gmres, eig=not args.no_eig,
                             oracle_leg=oracle_leg)
    shard = None
    if not args.no_shard:
        log("one GPU's share of an 8-way row decomposition")
        shard = shard_leg(ctx, xab, torch, gen, A)
    c4 = None
    if not args.no_batch:
        log("batch of 512 systems: batched SpMV and BiCGStab")
        c4 = batch_leg(ctx, xab, torch, gen)

    stress = trans4_leg(ctx, xab, torch, gen)
    c1 = None if args.no_c1 else c1_leg(ctx, xab, torch, gen)

    cpu, errs = None, {}
    if oracle_leg:
        log("waiting for the CPU oracle leg")
        cpu, errs = oracle_leg.join()
        if "powerlaw" in errs:
            fp32["error_per_result"] = errs["powerlaw"]
        if c3 is not None and "sym27" in errs:
            c3["error_per_result"] = errs["sym27"]

    out = {
        "metric": "SpMV GB/s & % HBM peak (FP64 vs FP32-val); GMRES s to 1e-10 residual",
        "value": round(gbs, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"power-law CSR n={A.n} nnz={A.nnz} (lognormal(2.5,1) rows), FP64 SpMV, "
                               "TIME-policy selected implementation", "n": A.n, "nnz": A.nnz,
                   "selected": plan.describe()},
        "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
        "cold_us_per_step": cold,
        "stream": dict(stream, frac_of_read=round(gbs / stream["read_gbs"], 4)),
        "xcb_gather_reference": gather_ref,
        "gflops": round(2 * A.nnz / (wall / args.steps) / 1e9, 1),
        "fp32_values": fp32,
        "selector": {"chosen_class": chosen, "us_per_class": times, "select_ms": round(float(info.select_ms), 2),
                     "select_wall_ms": round(time_wall_ms, 2), "learned": learned,
                     "plan_mb_per_class": plan_mb, "memory_policy": memory},
        "gmres": gm,
        "sym27": c3,
        "trans4_stress": stress,
        "c1_laplacian64": c1,
        "batch512": c4,
        "shard_of_8": shard,
        "arnoldi": arn,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
