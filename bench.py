"""Throughput of the transport step on one MI355X.

Workload: the high-resolution axisymmetric profile (600 r x 256 theta zones,
3 species, 24 logarithmic groups 2-300 MeV, 12 Gauss-Lobatto mu x 8 Phi =
96 directions, ~1.06e9 phase-space values) with seeded shock and l = 1-8
density perturbations, in mixed precision; the same grid is then stepped in
FP64 for the mixed-vs-FP64 speedup and the moment error of the mixed run.
Inputs are synthetic (paper_2003_02845_amd.workloads) and resident in HBM
before timing starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=["hires_2d", "shock_2d", "axisym_2d"], default="hires_2d",
                    help="hires_2d: the high-resolution grid (sizes from --n-r, --n-theta); shock_2d: "
                         "550 x 128 zones, 3 species, 21 groups, 10 x 8 directions; axisym_2d: 256 x 64 "
                         "zones, 1 species, 16 groups, 8 x 8 directions")
    ap.add_argument("--n-r", type=int, default=600)
    ap.add_argument("--n-theta", type=int, default=256)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--lts-level", type=int, default=6,
                    help="highest time level of the local-time-stepping run (0: skip it)")
    ap.add_argument("--lts-steps", type=int, default=2)
    ap.add_argument("--no-shard", dest="shard", action="store_false",
                    help="skip the timing of one GPU's share of a radially split grid")
    ap.add_argument("--evolve-steps", type=int, default=3,
                    help="steps of the run whose background changes every step (0: skip it)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--cpu-theta", type=int, default=256,
                    help="theta rows of the grid the CPU reference is timed on with all threads")
    ap.add_argument("--cpu-leg", nargs=2, type=int, metavar=("THREADS", "N_THETA"), default=None,
                    help=argparse.SUPPRESS)    # child process: one reference step, no GPU
    return ap.parse_args()


def device_state(torch, w, dtype):
    feq = torch.from_numpy(np.ascontiguousarray(w.f_eq)).cuda().to(dtype)
    return feq[..., None].expand(w.n_zones, w.n_species, w.n_eps, w.n_dir).contiguous()


def run_gpu(torch, btx, w, precision, steps, warmup):
    stream = torch.cuda.current_stream()
    ctx = btx.Context(w, device=0, stream=stream.cuda_stream, precision=precision)
    ctx.set_background()
    dtype = torch.float32 if precision == 1 else torch.float64
    f0 = device_state(torch, w, dtype)
    ctx.set_state(f0)
    del f0
    dt = ctx.max_dt(w.cfl)
    ctx.step(dt, warmup)
    torch.cuda.synchronize()
    ctx.timing(enable=True, reset=True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall = time.perf_counter()
    t0.record(stream)
    ctx.step(dt, steps)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall
    ms = t0.elapsed_time(t1)
    kms, kn = ctx.timing(enable=False, reset=True)
    zm, tot = ctx.moments()
    ctx.close()
    return {"ms": ms, "wall": wall, "kernel_ms": kms / np.maximum(kn, 1), "zm": zm, "tot": tot,
            "dt": dt}


def run_lts(torch, btx, w, max_level, steps, ref_ms_per_step):
    """the same grid and precision with time levels: each step is 2^L substeps of
    the global dt; reported as simulated time per second against the global step"""
    stream = torch.cuda.current_stream()
    ctx = btx.Context(w, device=0, stream=stream.cuda_stream, precision=1)
    ctx.set_background()
    f0 = device_state(torch, w, torch.float32)
    ctx.set_state(f0)
    del f0
    dt = ctx.max_dt(w.cfl)
    lev = ctx.time_levels(max_level)
    L = int(lev.max())
    ctx.set_time_levels(lev)
    ctx.step(dt, 1)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    ctx.step(dt, steps)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    _, tot = ctx.moments()
    ctx.close()
    zone_updates = float(np.sum(2.0 ** (L - lev)))
    sim_per_s = (2 ** L) * dt / (ms * 1e-3)
    sim_global = dt / (ref_ms_per_step * 1e-3)
    return {"max_level": L, "zones_per_level": np.bincount(lev, minlength=L + 1).tolist(),
            "ms_per_step": ms, "substeps_per_step": 2 ** L,
            "simulated_time_per_s": sim_per_s, "speedup_vs_global_step": sim_per_s / sim_global,
            "zone_update_fraction": zone_updates / (w.n_zones * 2 ** L),
            "updates_per_s": zone_updates * w.block / (ms * 1e-3)}


def run_evolving(torch, btx, w, steps, static_ms):
    """a background that changes every step (velocity, lapse, conformal factor,
    absorption): each step is a background update (the state remapped into the
    new comoving frames and the remap tables rebuilt) followed by one step;
    wall clock, mixed precision.  The backgrounds are FP64 arrays already in
    GPU memory (btx_update_background_device); the same with host arrays
    (btx_update_background, PCIe-inclusive) is reported beside it."""
    import copy
    stream = torch.cuda.current_stream()
    ctx = btx.Context(w, device=0, stream=stream.cuda_stream, precision=1)
    ctx.set_background()
    f0 = device_state(torch, w, torch.float32)
    ctx.set_state(f0)
    del f0
    dt = ctx.max_dt(w.cfl)
    bgs, dbgs = [], []
    for k in range(2):
        b = copy.copy(w)
        b.v_r = w.v_r * (1.0 + 0.01 * (k + 1))
        b.alpha = w.alpha * (1.0 - 0.001 * (k + 1))
        b.psi = b.alpha ** -0.5
        b.kappa_a = w.kappa_a * (1.0 + 0.01 * (k + 1))
        bgs.append(b)
        dbgs.append({n: torch.from_numpy(np.ascontiguousarray(getattr(b, n), float).reshape(-1)).cuda()
                     for n in ("v_r", "v_theta", "alpha", "psi", "kappa_a", "kappa_s", "f_eq")})
    out = {}
    for mode in ("device", "host"):
        upd = (lambda k: ctx.update_background_device(dbgs[k % 2])) if mode == "device" else \
              (lambda k: ctx.update_background(bgs[k % 2]))
        upd(1)
        ctx.step(dt, 1)
        torch.cuda.synchronize()
        t_upd = 0.0
        wall = time.perf_counter()
        for k in range(steps):
            torch.cuda.synchronize()                    # the update alone: the previous step done
            t = time.perf_counter()
            upd(k)                                      # synchronises the stream
            t_upd += time.perf_counter() - t
            ctx.step(dt, 1)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall
        out[mode] = {"ms_per_step": wall / steps * 1e3, "update_ms": t_upd / steps * 1e3,
                     "updates_per_s": w.n_values * steps / wall,
                     "vs_static_step": wall / steps * 1e3 / static_ms}
    ctx.close()
    res = dict(out["device"])
    res["background_in"] = "GPU memory (btx_update_background_device)"
    res["host_arrays"] = out["host"]
    return res


def cpu_leg(threads, n_theta):
    """child process of cpu_baseline: one FP64 reference step of the benchmark profile on
    n_theta theta rows with the given OpenMP thread count (set in its environment); no GPU"""
    from oracle import oracle
    from paper_2003_02845_amd import workloads as W
    w = W.hires_2d(n_theta=n_theta)
    o = oracle.Oracle(w)
    dt = o.max_dt(w.cfl)
    t = time.perf_counter()
    o.step(dt, 1)
    el = time.perf_counter() - t
    print(json.dumps({"seconds": el, "values": w.n_values, "threads": threads,
                      "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_theta):
    """the CPU reference (oracle) on the host cores: one FP64 step of the benchmark grid
    (n_theta theta rows; 256 is the whole grid) with every thread the process may use, and
    one step of an 8-row slice of it on one thread.  Each runs in a child process that
    touches no GPU, so its OpenMP thread count is set before the library loads."""
    import subprocess
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = int(os.environ.get("OMP_NUM_THREADS", avail))
    def leg(nt, rows):
        env = dict(os.environ, OMP_NUM_THREADS=str(nt), OMP_PROC_BIND="false")
        try:
            res = subprocess.run([sys.executable, "-u", os.path.abspath(__file__), "--cpu-leg", str(nt), str(rows)],
                                 env=env, capture_output=True, text=True, timeout=900)
        except subprocess.TimeoutExpired:
            return None
        if res.returncode != 0:
            print(f"[bench] cpu leg ({nt} threads, {rows} rows) failed: {res.stderr[-500:]}", file=sys.stderr,
                  flush=True)
            return None
        r = json.loads(res.stdout.strip().splitlines()[-1])
        print(f"[bench] cpu: {nt} thread(s), {rows} theta rows: {r['seconds']:.1f} s", file=sys.stderr, flush=True)
        return r
    # the whole grid needs about 90 GB of host memory; a quarter of it if that fails
    full = leg(threads, n_theta)
    if full is None and n_theta > 64:
        n_theta = 64
        full = leg(threads, n_theta)
    one = leg(1, 8)
    if full is None or one is None:
        return {"value": None, "unit": "zone*group*direction updates/s", "cores": threads, "kind": "oracle",
                "sample": "the CPU reference legs did not complete", "cpu_model": cpu_model()}
    return {"value": full["values"] / full["seconds"], "unit": "zone*group*direction updates/s",
            "cores": threads, "kind": "oracle",
            "sample": f"one FP64 step of the benchmark grid, 600 r x {n_theta} theta zones "
                      f"({full['values']:.4g} values, {full['seconds']:.1f} s on {threads} threads)",
            "cpu_model": cpu_model(), "cpus_available": avail,
            "value_1thread": one["values"] / one["seconds"],
            "sample_1thread": f"one FP64 step of 600 r x 8 theta zones of the same profile "
                              f"({one['values']:.4g} values, {one['seconds']:.1f} s on 1 thread)"}


def run_batch(torch, btx, W, steps):
    """the 64-model batch of spherically symmetric models (mixed precision): one batched,
    graph-replayed step against 64 sequential single-model steps, same models and dt"""
    ws = W.batch_models()
    stream = torch.cuda.current_stream()
    b = btx.Batch(ws, precision=W.PREC_MIXED, stream=stream.cuda_stream)
    for m, w in enumerate(ws):
        b.set_background(m)
        b.set_state(m, w.f0)
    dts = [b.max_dt(m, 0.4) for m in range(len(ws))]
    b.step(dts, 2)                                  # tuning, graph capture, warm-up
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    b.step(dts, steps)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_b = t0.elapsed_time(t1) / steps
    shapes = sorted({f"{a}x{c}" for a, c in (b.shape(m) for m in range(len(ws)))})
    # the same batch with time levels (up to 4 per model): 2^L substeps a step
    levs = [b.time_levels(m, 4) for m in range(len(ws))]
    for m in range(len(ws)):
        b.set_time_levels(m, levs[m])
    L = max(int(l.max()) for l in levs)
    b.step(dts, 1)
    torch.cuda.synchronize()
    lts_steps = max(1, steps // (2 ** L))
    t0.record(stream)
    b.step(dts, lts_steps)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_l = t0.elapsed_time(t1) / lts_steps
    b.close()
    ctxs = []
    for m, w in enumerate(ws):
        c = btx.Context(w, precision=W.PREC_MIXED, stream=stream.cuda_stream)
        c.set_background()
        c.set_state(w.f0)
        c.step(dts[m], 1)
        ctxs.append(c)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(steps):
        for m, c in enumerate(ctxs):
            c.step(dts[m], 1)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_s = t0.elapsed_time(t1) / steps
    for c in ctxs:
        c.close()
    nv = sum(w.n_values for w in ws)
    return {"workload": "64 spherically symmetric models, 100-600 radial zones, 12-24 groups, "
                        "16-48 directions, mixed precision",
            "values": nv, "steps": steps, "ms_per_step": ms_b, "value": nv / (ms_b * 1e-3),
            "sequential_ms_per_step": ms_s, "sequential_value": nv / (ms_s * 1e-3),
            "speedup_vs_sequential": ms_s / ms_b, "face_shapes": shapes,
            "time_levels": {"max_level": L, "ms_per_step": ms_l, "substeps_per_step": 2 ** L,
                            "speedup_vs_global_step": (2 ** L) * ms_b / ms_l}}


def kernel_source_hash():
    """sha256 (first 16 hex) over the library's sources (csrc/, in name order): a counter
    summary applies only to the kernels it was taken from"""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2003_02845_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def profile_values(name):
    """key -> value lines ('# key value') of a committed counter summary under profiles/, or
    None when the summary is missing or was taken from other kernel sources"""
    try:
        text = open(os.path.join(ROOT, "profiles", name)).read()
    except OSError:
        return None
    m = re.search(r"kernel sources sha256 \(first 16 hex\): ([0-9a-f]{16})", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    return {k: float(v) for k, v in re.findall(r"^# ([a-z0-9_]+) ([-0-9.e+]+)$", text, re.M)}


def main():
    a = parse()
    if a.cpu_leg is not None:
        cpu_leg(*a.cpu_leg)
        return
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              f"(the spatial decomposition across GPUs is a design, not a build)", file=sys.stderr)
        sys.exit(2)
    cpu = None if a.no_cpu else cpu_baseline(a.cpu_theta)    # before this process touches the GPU
    import torch
    from paper_2003_02845_amd import btx, workloads as W
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    w = W.hires_2d(n_r=a.n_r, n_theta=a.n_theta) if a.workload == "hires_2d" else getattr(W, a.workload)()
    full = a.workload == "hires_2d" and (a.n_r, a.n_theta) == (600, 256)
    print(f"[bench] workload {w.name}: {w.n_zones} zones x {w.block} = {w.n_values:.4g} values",
          file=sys.stderr, flush=True)
    mixed = run_gpu(torch, btx, w, W.PREC_MIXED, a.steps, a.warmup)
    upd = w.n_values * a.steps
    value = upd / (mixed["ms"] * 1e-3)
    print(f"[bench] mixed: {mixed['ms'] / a.steps:.3f} ms/step, {value:.4g} updates/s, "
          f"kernels {mixed['kernel_ms']}", file=sys.stderr, flush=True)
    res64 = None
    if not a.no_fp64:
        k64 = a.fp64_steps if a.fp64_steps is not None else a.steps
        res64 = run_gpu(torch, btx, w, W.PREC_FP64, k64, a.warmup)
        v64 = w.n_values * k64 / (res64["ms"] * 1e-3)
        print(f"[bench] fp64: {res64['ms'] / k64:.3f} ms/step, {v64:.4g} updates/s, "
              f"kernels {res64['kernel_ms']}", file=sys.stderr, flush=True)
    if a.copy_probe:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
    # algorithmic bytes of a step (mixed): f read and written once (4 B each), ka, ks, feq per
    # (zone, species, group) (FP32) and v_r, v_theta, alpha, psi per zone (FP64)
    nz, nsg = w.n_zones, w.n_zones * w.n_species * w.n_eps
    b_step = w.n_values * 8 + nsg * 3 * 4 + nz * 4 * 8
    # the face kernel's own share: f and the opacities read once
    b_face = w.n_values * 4 + nsg * 3 * 4 + nz * 4 * 8
    t_face = mixed["kernel_ms"][0] * 1e-3
    achieved = b_step / t_face / 1e9
    # the zone kernel: f read and written, the opacities and the zone background
    b_zone = w.n_values * 8 + nsg * 3 * 4 + nz * 4 * 8
    t_zone = mixed["kernel_ms"][1] * 1e-3
    hbm = profile_values("face_kernel_hires_2d_mixed_hbm_traffic.txt") if full else None
    alu = profile_values("face_kernel_hires_2d_mixed_valu_lds.txt") if full else None
    compute = None
    if alu is not None:
        # VALU issue: one wave64 instruction per CU per cycle (4 SIMDs, 4 cycles each)
        peak_inst = 256 * 2.4e9
        inst_rate = alu["valu_insts_per_launch"] / t_face
        compute = {"bound": "alu", "kernel": "face_kernel<float>",
                   "achieved": inst_rate / 1e9, "peak": peak_inst / 1e9, "unit": "G wave-VALU instr/s",
                   "frac": inst_rate / peak_inst,
                   "valu_busy": alu["valu_busy_pct"] / 100.0,
                   "lds_bank_conflict_of_lds_cycles": alu["lds_bank_conflict_pct_of_lds_active"] / 100.0,
                   "lds_busy": alu["lds_active_pct"] / 100.0,
                   "waves_per_cu": alu["mean_waves_per_cu"],
                   "fp32_flops_est": {"per_update": 350, "achieved_tflops": 350 * w.n_values / t_face / 1e12,
                                      "peak_tflops": 157.3,
                                      "frac": 350 * w.n_values / t_face / 1e12 / 157.3},
                   "source": "profiles/face_kernel_hires_2d_mixed_valu_lds.txt (rocprofv3 --pmc, full size)"}
    out = {
        "metric": "zone\u00b7group\u00b7direction updates/s, mixed FP32/FP64 vs FP64; % HBM peak",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": mixed["ms"] / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n_r} r x {w.n_theta} theta zones, {w.n_species} species, "
                               f"{w.n_eps} groups, {w.n_mu} mu x {w.n_phi} Phi directions, mixed precision",
                   "zones": nz, "values": w.n_values, "dt": mixed["dt"]},
        "step_hbm_frac": b_step / (mixed["ms"] / a.steps * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "kernel": "face_kernel<float>", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if hbm is None else hbm["face_traffic_bytes"] / 1e9,
                     "traffic_unit": "GB per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic": b_step / 1e9,
                     "algorithmic_unit": "GB per launch: the step's algorithmic bytes (f read and written "
                                         "once, opacities, background) over the dominant kernel's time",
                     "face_only": {"algorithmic": b_face / 1e9, "achieved": b_face / t_face / 1e9,
                                   "frac": b_face / t_face / 1e9 / HBM_PEAK_GBS}},
        "compute_roofline": compute,
        "zone_roofline": {"bound": "hbm", "kernel": "zone_kernel<float>", "achieved": b_zone / t_zone / 1e9,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": b_zone / t_zone / 1e9 / HBM_PEAK_GBS,
                          "traffic": None if hbm is None else hbm["zone_traffic_bytes"] / 1e9,
                          "traffic_rate": None if hbm is None else hbm["zone_traffic_bytes"] / t_zone / 1e9,
                          "traffic_unit": "GB per launch; GB/s",
                          "algorithmic": b_zone / 1e9, "algorithmic_unit": "GB per launch"},
    }
    if res64 is not None:
        k64 = a.fp64_steps if a.fp64_steps is not None else a.steps
        v64 = w.n_values * k64 / (res64["ms"] * 1e-3)
        out["fp64_value"] = v64
        out["speedup_vs_fp64"] = value / v64
        # moment error of the mixed run against the FP64 GPU run (same steps only if equal)
        if k64 == a.steps:
            zm, z64 = mixed["zm"], res64["zm"]
            J64 = z64[..., 1]
            mask = np.abs(J64) > 1e-8 * np.abs(J64).max()
            out["mixed_vs_fp64_rel_err"] = {
                "N": float(np.max(np.abs(zm[..., 0] - z64[..., 0])[mask] / np.abs(z64[..., 0][mask]))),
                "J": float(np.max(np.abs(zm[..., 1] - J64)[mask] / np.abs(J64[mask])))}
        tot = mixed["tot"]
        if k64 == a.steps:
                out["number_drift_mixed"] = float(np.max(np.abs(tot[:, 0] + tot[:, 1] - res64["tot"][:, 0]
                                                            - res64["tot"][:, 1]) / res64["tot"][:, 0]))
    if a.shard:
        # one GPU's share of the grid split radially over 8 GPUs: 75 radial
        # zones (plus the two-zone halos on each side) of every theta row
        n_own = w.n_r // 8
        slab = W.radial_slab(w, 3 * n_own - 2, n_own + 4)
        sh = run_gpu(torch, btx, slab, W.PREC_MIXED, a.steps, a.warmup)
        out["shard"] = {"workload": f"radial slab of {n_own} + 2 x 2 halo zones x {w.n_theta} theta rows "
                                    f"(one eighth of the grid), mixed precision",
                        "ms_per_step": sh["ms"] / a.steps,
                        "updates_per_s": slab.n_values * a.steps / (sh["ms"] * 1e-3),
                        "owned_updates_per_s": n_own * w.n_theta * w.block * a.steps / (sh["ms"] * 1e-3)}
        print(f"[bench] shard: {out['shard']['ms_per_step']:.3f} ms/step for {slab.n_zones} zones",
              file=sys.stderr, flush=True)
    if a.lts_level > 0:
        out["local_time_stepping"] = run_lts(torch, btx, w, a.lts_level, a.lts_steps, mixed["ms"] / a.steps)
        l = out["local_time_stepping"]
        print(f"[bench] time levels (max {l['max_level']}): {l['ms_per_step']:.2f} ms per "
              f"{l['substeps_per_step']} substeps, {l['speedup_vs_global_step']:.2f}x the simulated time "
              f"per second of the global step", file=sys.stderr, flush=True)
    if a.evolve_steps > 0:
        out["evolving_background"] = run_evolving(torch, btx, w, a.evolve_steps, mixed["ms"] / a.steps)
        e = out["evolving_background"]
        print(f"[bench] evolving background: {e['ms_per_step']:.1f} ms per step ({e['vs_static_step']:.2f}x "
              f"the static step), of which {e['update_ms']:.1f} ms background update from GPU arrays; "
              f"from host arrays {e['host_arrays']['ms_per_step']:.1f} ms, update "
              f"{e['host_arrays']['update_ms']:.1f} ms", file=sys.stderr, flush=True)
    if not a.no_batch:
        out["batch"] = run_batch(torch, btx, W, a.batch_steps)
        bt = out["batch"]["time_levels"]
        print(f"[bench] batch: {out['batch']['ms_per_step']:.3f} ms/step batched, "
              f"{out['batch']['sequential_ms_per_step']:.3f} ms/step sequential; with time levels "
              f"(max {bt['max_level']}) {bt['ms_per_step']:.3f} ms per {bt['substeps_per_step']} substeps, "
              f"{bt['speedup_vs_global_step']:.2f}x the simulated time per second", file=sys.stderr, flush=True)
    if cpu is not None:
        out["cpu_baseline"] = cpu
        if cpu["value"]:
            out["cpu_baseline"]["gpu_speedup"] = value / cpu["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
