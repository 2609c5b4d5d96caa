#!/usr/bin/env python3
"""Throughput of HHFFBPA against direct backprojection on one MI355X.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu-baseline]
                    [--workload large|mid|autofocus|paper_sim]

Default workload ("HHFFBPA large"): 65536 handheld positions (44 serpentine
strokes over 0.3 x 0.3 m plus 20 persistent walks in the central 80 mm,
0.5-3.7 samples/mm^2), 128 frequencies 24-40 GHz, a 256x256x128 voxel grid at
1 mm centred 0.3 m in front of the aperture, 200 point targets and a
5000-scatterer slab of complex-normal amplitudes; float32 (complex64) storage.
The timed form: HHFFBPA with 4 merge stages of factor 4 onto a compressed root
grid with one resample to the voxels, band-limited interpolation weights on
grids oversampled (2.2, 2.2, 2.6), range profiles at 4-fold range oversampling
read by linear interpolation.  The mid workload (16384 positions, 64 f,
128x128x64 voxels, 3 stages onto the voxel grid) is reported beside it.

A step is one hhffbp_image call: range compression, level-1 backprojection, the
merges and the final resample, with the echoes already resident in device
memory.  The metric counts voxel x position backprojections: N_vox * N_pos per
step (the direct-BP work that HHFFBPA replaces).  Plan construction (host) is
timed separately (``plan_ms``).  Beside the timed form: the ES parity mode on the
same grids, half and bfloat16 storage, and the direct-BP baseline (the fastest
linear-kernel direct mode within -30 dB of the ES direct image) and eq. (4)
itself.  Errors are NRMSE against GPU ES direct BP on the full grid (itself
<= 1e-5 of float64 eq. (4)) and, for the large workload, against float64 eq. (4)
on the stored stratified voxel sample.  One JSON line is printed.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel·position backprojections/s, HHFFBPA vs direct BP on 1 GPU at ≤−30 dB NRMSE"
BL_GAMMA = (2.2, 2.2, 2.6)       # band-limited interpolation grids (the timed form)
BL_LEAF = (1.8, 1.8, 2.2)        # ... its level-1 (leaf) grids
BENCH_U = 4.0                    # range oversampling of its linear range kernel
DIRECT_U = (2.0, 3.0, 4.0, 8.0)  # linear-kernel direct-BP candidates for the baseline
AF_GAMMA = BL_GAMMA              # band-limited grids of the autofocus workload
AF_LEAF = BL_LEAF                # ... its leaf grids
TAPS = 4
# the timed form per workload index: stages and root grid
TIMED = {2: dict(stages=4, root_grid=True, oversample_leaf=BL_LEAF),
         1: dict(stages=3, root_grid=False, oversample_leaf=BL_LEAF)}
WORKLOAD_NAME = {
    2: "HHFFBPA large: 65536 handheld positions (44 serpentine strokes + 20 dense walks, "
       "0.5-3.7 samples/mm^2), 128 f 24-40 GHz, 256x256x128 voxels at 1 mm, 200 points + "
       "5000-scatterer slab at 0.33 m",
    1: "HHFFBPA mid: 16384 handheld positions (64 serpentine strokes, 0.3x0.3 m), 64 f "
       "24-40 GHz, 128x128x64 voxels at 1.5 mm, 50 points + 10x10x10 cube at 0.3 m",
}
# Peaks of MI355X (256 CUs at 2.4 GHz): VALU issue 256 x 4 SIMD x 16 lanes x 2.4 GHz
# lane-ops/s (packed FP32 disabled, every VALU op one lane-op); FP32 MFMA
# 157.3 TFLOP/s; vector L1 64 B/clk/CU; HBM 8 TB/s.
VALU_PEAK_OPS = 256 * 64 * 2.4e9
MFMA_F32_PEAK = 157.3e12
MFMA_BF16_PEAK = 2.5e15  # dense
L1_PEAK_BPS = 256 * 64 * 2.4e9
HBM_PEAK_BPS = 8.0e12
# Algorithmic VALU lane-ops per (leaf grid point, position) backprojection in
# the cancellation-free range-compressed form, the fewest this evaluation
# needs: the distance-difference numerator num = |d|^2 - 2 q.d 3 FMA,
# |q - p'| = sqrt(|q - c|^2 + num) 2, Delta R = num / (|q - p'| + |q - c|) 3
# (add, reciprocal, multiply), bin coordinate 3 (FMA, floor to int, fraction),
# tap address 1, carrier 3 (scale to turns, sin, cos), complex accumulate 4;
# the range read: linear kernel v0 + x (v1 - v0) per component 4, or the 7-tap
# ES kernel with 6 per weight and 2 per tap sum.
LEAF_OPS_LINEAR = 3 + 2 + 3 + 3 + 1 + 3 + 4 + 4
LEAF_OPS_ES = 3 + 2 + 3 + 3 + 1 + 3 + 4 + (6 + 2) * 7
# Algorithmic VALU lane-ops per (point, child) interpolation of a merge or the
# final stage (T = 4, band-limited weights, geometry from the plan's records):
# weights 54 (per axis y = x - 1/2, y^2, two 3-FMA Horner chains per tap pair
# and the even/odd combination), taps 168 (64 x 2 FMA along n, 16 x 2 FMA
# along v, 4 x 2 FMA along u), rotation by the pair's phase 6 (sin, cos, 4 FMA).
INTERP_OPS_PER_PAIR = 54 + 168 + 6
KERNEL_SOURCES = ("kernels.hip", "device_common.hpp", "hhffbp_internal.hpp")
TRAFFIC_SUMMARY = "hhffbp_large_hbm_traffic.md"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_description():
    """nproc, the usable cores and the CPU model of this host."""
    out = {"nproc": os.cpu_count(), "usable_cores": len(os.sched_getaffinity(0))}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core",
                             "CPU(s)"):
                out[k.strip()] = v.strip()
    except Exception:
        pass
    return out


def oracle_cpu_baseline(w, index, target_s=12.0):
    """The float64 oracle on the host cores: eq. (4) on voxels of the stored
    stratified sample (large: the point targets' boxes and seeded uniform voxels
    of tests/golden/large_oracle.npz; mid: seeded voxels), on all the threads the
    oracle uses and on one; and the oracle HHFFBPA on one 4x4x4 voxel brick,
    through the cone of grid points its stencils reach (oracle.hhffbp.image_at)."""
    import numpy as np

    from oracle import hhffbp as OH
    from oracle import native
    from oracle import plan as OP
    from workloads import voxel_centres

    vox = voxel_centres(w.grid_origin, w.grid_pitch, w.grid_dims)
    if index == 2:
        pool = np.load(os.path.join(ROOT, "tests", "golden", "large_oracle.npz"))["index"]
        what = "the stored stratified sample (target boxes + seeded uniform voxels)"
    else:
        pool = np.arange(vox.shape[0])
        what = "seeded voxels"
    rng = np.random.default_rng(3)
    cores = native._nthreads()
    n = 8
    while True:
        sel = rng.choice(pool, n, replace=False)
        t = time.time()
        OH.direct_bp(w.positions, w.freqs_hz, w.echoes, vox[sel])
        dt = time.time() - t
        if dt >= 1.5 or n >= pool.size:
            break
        n = min(pool.size, 4 * n)
    n2 = int(min(pool.size, max(n, round(n * target_s / max(dt, 1e-3)))))
    sel = rng.choice(pool, n2, replace=False)
    t = time.time()
    OH.direct_bp(w.positions, w.freqs_hz, w.echoes, vox[sel])
    dt = time.time() - t
    n1 = int(max(8, min(pool.size, round(n2 / cores / 3))))
    sel1 = rng.choice(pool, n1, replace=False)
    k = 2.0 * np.pi * np.asarray(w.freqs_hz, float) / 299792458.0
    t = time.time()
    native.bp_eq4(w.positions, k, w.echoes, vox[sel1], nthreads=1)
    dt1 = time.time() - t
    # the oracle HHFFBPA (timed form's grid choices, S = 3 onto the voxel grid) on
    # one brick of 64 voxels at the grid centre
    t = time.time()
    op = OP.build_plan(w.positions, w.freqs_hz, w.grid_origin, w.grid_pitch, w.grid_dims, 3, 4,
                       BL_GAMMA, TAPS, kernel="bandlimited")
    plan_s = time.time() - t
    d = np.asarray(w.grid_dims)
    c = d // 2 - 2
    r = np.arange(4)
    bx = [((c[0] + a) * d[1] + c[1] + b) * d[2] + c[2] + e for a in r for b in r for e in r]
    t = time.time()
    OH.image_at(op, w.echoes, w.positions, np.array(bx), range_u=BENCH_U)
    dth = time.time() - t
    return {"value": n2 * w.n_pos / dt, "unit": "vp/s", "cores": cores, "kind": "oracle",
            "sample": f"float64 eq. (4) on {n2} voxels of {what} x {w.n_pos} positions x "
                      f"{w.n_f} frequencies ({dt:.1f} s)",
            "value_1thread": n1 * w.n_pos / dt1,
            "sample_1thread": f"{n1} voxels of the same sample on one thread ({dt1:.1f} s)",
            "hhffbp_oracle": {"value": 64 * w.n_pos / dth, "unit": "vp/s", "seconds": dth,
                              "plan_seconds": plan_s,
                              "sample": "oracle HHFFBPA (S=3, band-limited (2.2, 2.2, 2.6), "
                                        "linear U=4) on one 4x4x4 voxel brick through its "
                                        "stencil cone; a cone does not amortise the level-1 "
                                        "sums over the image as a whole image does"},
            "host": host_description()}


def kernel_source_hash():
    """sha256 over the code of the sources that make up the imaging kernels:
    comments and whitespace are left out, so that editing a comment does not
    discard the measured traffic of unchanged code."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2506_23568_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter
    summary, or None when it is missing or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic_json:"):
                rec = json.loads(line[len("traffic_json:"):])
                if rec.get("source_sha256") != kernel_source_hash():
                    return None
                k = rec.get("kernels", {}).get(kernel)
                return None if k is None else k["bytes_per_launch"]
    return None


def copy_probe(torch, mib):
    """One plain device copy of ``mib`` MiB (scale reference for HBM counters)."""
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def autofocus_report(args):
    """Autofocus workload: the large scene imaged at positions with a smooth
    trajectory error; 20 Adam steps on a 16-mode cosine motion model of the
    positions through forward, loss and backward kernels, for each
    half-precision storage form."""
    import numpy as np
    import torch

    import paper_2506_23568_amd as H
    from paper_2506_23568_amd.autofocus import autofocus
    from workloads import make_config

    log("synthesising the autofocus workload (float64 sums on the GPU)")
    w = make_config(4, synth_device="cuda")
    p_img = w.imager_positions
    a3 = (p_img, w.freqs_hz, w.grid_origin, w.grid_pitch, w.grid_dims)
    kw = dict(stages=args.af_stages, merge_factor=4, oversample=AF_GAMMA, oversample_leaf=AF_LEAF,
              interp_taps=TAPS,
              interp_kernel="bandlimited")
    if args.af_range == "linear":
        kw.update(range_kernel="linear", range_oversample=args.af_u)
    if args.af_root_grid == "on":
        kw.update(root_grid=True)
    pos_true = torch.from_numpy(w.positions).cuda()
    pos0 = torch.from_numpy(p_img.copy()).cuda()
    ech64 = torch.from_numpy(w.echoes.astype(np.complex64)).cuda()
    pd = H.Plan(*a3, mode="direct_rc")
    ref = pd.image(ech64, positions=pos_true)   # clean-trajectory direct BP (float32, ES)
    clean = H.Plan(*a3, **kw).image(ech64, positions=pos_true)
    nref = torch.linalg.norm(ref)
    out = {}
    work = None
    for storage in ("f16", "bf16"):
        pl = H.Plan(*a3, storage=storage, **kw)
        if work is None:
            info = pl.info()
            work = {k: info[k] for k in ("leaf_pairs", "merge_pairs", "final_pairs")}
        ech = H.Plan.pack_echoes(torch.from_numpy(w.echoes), storage).cuda()
        e0 = (torch.linalg.norm(pl.image(ech, positions=pos0) - ref) / nref).item()
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        pos, hist = autofocus(pl, ech, pos0, steps=args.steps, clean=clean)
        peak = torch.cuda.max_memory_allocated() + pl.info()["device_bytes"]
        e1 = (torch.linalg.norm(pl.image(ech, positions=pos) - ref) / nref).item()
        ms = float(np.median([h["ms"] for h in hist[1:]]))
        out[storage] = {
            "ms_per_step": ms, "peak_device_bytes": int(peak),
            "loss_first": hist[0]["loss"], "loss_last": hist[-1]["loss"],
            "nrmse_vs_clean_direct_db_start": 20 * np.log10(e0),
            "nrmse_vs_clean_direct_db_end": 20 * np.log10(e1),
            "mean_position_error_mm_start": (pos0 - pos_true).norm(dim=1).mean().item() * 1e3,
            "mean_position_error_mm_end": (pos - pos_true).norm(dim=1).mean().item() * 1e3,
        }
        log(f"{storage}: {out[storage]}")
    steps_s = args.steps / (out["f16"]["ms_per_step"] * args.steps * 1e-3)
    print(json.dumps({
        "metric": "autofocus steps/s (forward + loss + backward + Adam), half storage",
        "loss": "relative L2 distance to the clean-trajectory HHFFBPA image (float32 storage)",
        "value": steps_s, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": 0,
        "ms_per_step": out["f16"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f16 storage, f32 arithmetic", "data": "synthetic",
        "config": {"workload": "autofocus: 65536 positions (44 strokes + 20 dense walks), 128 f "
                               "24-40 GHz, 256x256x128 voxels at 1 mm, 200 points + 5000-scatterer "
                               f"slab, smooth trajectory error, S={args.af_stages} Q=4, 20 Adam steps (lr 0.03 mm) on 16 cosine modes per axis, relative-L2 loss to the clean-trajectory image",
                   "range_kernel": f"linear U={args.af_u:g}" if args.af_range == "linear" else "ES U=2 W=7",
                   "interp_kernel": "bandlimited", "oversample": list(AF_GAMMA),
                   "oversample_leaf": list(AF_LEAF),
                   "root_grid": args.af_root_grid == "on", "parallelism": "single GPU"},
        "storage": out, "work": work,
        "reference": "float32 direct BP (ES U=2 W=7) at the true positions, full grid"}), flush=True)


def paper_sim_report(args):
    """The shape of the paper's point-target simulation (Sec. V-A): 10201 positions
    of a jittered linear-array sweep, 24 f 12-15 GHz, 3x3x3 points, 101x101x51
    voxels; HHFFBPA and direct BP timed on one GPU, PSNR and the point-response
    metrics of the centre and squint scatterers."""
    import numpy as np
    import torch

    import paper_2506_23568_amd as H
    from paper_2506_23568_amd import psf
    from workloads import make_config

    w = make_config(5)
    a3 = (w.positions, w.freqs_hz, w.grid_origin, w.grid_pitch, w.grid_dims)
    ech = torch.from_numpy(w.echoes.astype(np.complex64)).cuda()
    gamma = (4.0, 4.0, 4.0)
    stream = torch.cuda.current_stream()

    def timed(plan, n, positions=None):
        img = plan.image(ech)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            plan.image(ech, out=img)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n, img

    d_ms, ref = timed(H.Plan(*a3, mode="direct_rc", range_kernel="linear", range_oversample=8.0), 3)
    _, ref_es = timed(H.Plan(*a3, mode="direct_rc"), 1)
    r = ref_es.cpu().numpy()
    out = {}
    for name, kw in (("fast", dict(range_kernel="linear", range_oversample=8.0)), ("es", {})):
        t = time.time()
        pl = H.Plan(*a3, stages=3, oversample=gamma, interp_taps=TAPS, **kw)
        plan_ms = (time.time() - t) * 1e3
        ms, img = timed(pl, args.steps)
        a = img.cpu().numpy()
        cuts = {}
        for label, c in (("centre", (0.0, 0.0, 0.4)), ("squint", (-0.175, 0.0, 0.4))):
            n = 401
            origin = np.array([c[0] - 0.05, c[1], c[2]])
            x = origin[0] + 0.25e-3 * np.arange(n)
            cp = H.Plan(w.positions, w.freqs_hz, origin, (0.25e-3, 1e-3, 1e-3), (n, 1, 1), stages=3,
                        oversample=gamma, interp_taps=TAPS, **kw)
            cd = H.Plan(w.positions, w.freqs_hz, origin, (0.25e-3, 1e-3, 1e-3), (n, 1, 1),
                        mode="direct_rc")
            mh = psf.psf_metrics(x, cp.image(ech).cpu().numpy().ravel())
            md = psf.psf_metrics(x, cd.image(ech).cpu().numpy().ravel())
            cuts[label] = {"hhffbp": {"mainlobe_mm": mh[0] * 1e3, "pslr_db": mh[1], "islr_db": mh[2]},
                           "direct_bp": {"mainlobe_mm": md[0] * 1e3, "pslr_db": md[1], "islr_db": md[2]}}
        out[name] = {"ms": ms, "vp_per_s": w.n_vox * w.n_pos / (ms * 1e-3), "plan_ms": plan_ms,
                     "nrmse_vs_direct_db": float(20 * np.log10(np.linalg.norm(a - r) / np.linalg.norm(r))),
                     "psnr_vs_direct_db": psf.psnr_db(a, r), "psf": cuts}
        log(f"{name}: {out[name]}")
    print(json.dumps({
        "metric": "voxel·position backprojections/s, HHFFBPA on the paper's simulation geometry",
        "value": out["fast"]["vp_per_s"], "unit": "vp/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": out["fast"]["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "paper-geometry simulation: 101-element linear array x 101 sweep "
                               "positions (0.45 m, depth fluctuation 6.5 cm), 24 f 12-15 GHz, 3x3x3 "
                               "points at 0.175 m around (0, 0, 0.4 m), 101x101x51 voxels over 0.5 m^3, "
                               "S=3 Q=4 gamma=(4,4,4) T=4", "parallelism": "single GPU"},
        "hhffbp": out,
        "direct_bp": {"ms": d_ms, "vp_per_s": w.n_vox * w.n_pos / (d_ms * 1e-3), "mode": "linear U=8"},
        "paper_context": {"hardware": "Ryzen 9 7950X, one thread (Sec. V-A)",
                          "bpa_s": 187.52, "hhffbpa_s": 3.02, "table": "III"}}), flush=True)


def imaging_report(args, index):
    """The imaging benchmark on workload ``index`` (2: large, 1: mid); returns
    the JSON record (see the module docstring)."""
    import numpy as np
    import torch

    import paper_2506_23568_amd as H
    from workloads import make_config

    log(f"synthesising workload {index} (float64 sums on the GPU)")
    w = make_config(index, synth_device="cuda")
    args3 = (w.positions, w.freqs_hz, w.grid_origin, w.grid_pitch, w.grid_dims)
    dev = torch.device("cuda:0")
    ech = torch.from_numpy(w.echoes.astype(np.complex64)).to(dev)
    stream = torch.cuda.current_stream(dev)
    vp = w.n_vox * w.n_pos
    form = dict(merge_factor=4, oversample=BL_GAMMA, interp_taps=TAPS, interp_kernel="bandlimited",
                **TIMED[index])

    def timed(plan, e, steps, warmup):
        """(ms per image over ``steps`` calls, per-stage ms, image).  The timed
        region holds the images alone; the per-stage times come from the same
        number of images right after it, with a HIP event on the launch stream
        after each stage (events between the kernels cost ~5 us each, so they
        stay out of the timed region)."""
        ws = plan._workspace(torch)
        img = torch.empty(w.grid_dims, dtype=torch.complex64, device=dev)
        for _ in range(warmup):
            plan.image(e, out=img, workspace=ws)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            plan.image(e, out=img, workspace=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        if args.only_timed:
            return ms, {}, img
        plan.profile_begin(steps)
        for _ in range(steps):
            plan.image(e, out=img, workspace=ws)
        torch.cuda.synchronize()
        st = plan.profile_end()
        return ms, {k: v[0] / max(v[1], 1) for k, v in st.items()}, img

    t = time.time()
    plan = H.Plan(*args3, range_kernel="linear", range_oversample=BENCH_U, **form)
    plan_ms = (time.time() - t) * 1e3
    info = plan.info()
    log("warm-up and timed steps")
    ms, kernels_ms, img = timed(plan, ech, args.steps, args.warmup)
    value = vp / (ms * 1e-3)
    rec = {
        "metric": METRIC, "value": value, "unit": "vp/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_NAME[index], "n_pos": w.n_pos, "n_freq": w.n_f,
                   "grid": list(w.grid_dims), "merge_factor": 4, "oversample": list(BL_GAMMA),
                   "interp_taps": TAPS, "interp_kernel": "bandlimited", "range_kernel": "linear",
                   "range_oversample": BENCH_U, "storage": "c64", "parallelism": "single GPU",
                   **TIMED[index]},
        "plan_ms": plan_ms, "kernels_ms": kernels_ms,
        "work": {"leaf_pairs": info["leaf_pairs"], "merge_pairs": info["merge_pairs"],
                 "final_pairs": info["final_pairs"], "level_points": info["level_points"],
                 "n_range_bins": info["n_range_bins"], "plan_device_bytes": info["device_bytes"]},
    }
    if args.only_timed:
        return rec

    log("references: ES direct BP (full grid) and the float64 sample")
    ref = H.Plan(*args3, mode="direct_rc", range_kernel="es", range_oversample=2.0,
                 range_taps=7).image(ech)
    torch.cuda.synchronize()
    nref = torch.linalg.norm(ref)
    sample = None
    if index == 2:
        g = np.load(os.path.join(ROOT, "tests", "golden", "large_oracle.npz"))
        sample = (torch.from_numpy(g["index"]).to(dev), g["bp"])

    def errors(im):
        out = {"nrmse_vs_direct_db": 20 * np.log10((torch.linalg.norm(im - ref) / nref).item())}
        if sample is not None:
            s = im.reshape(-1)[sample[0]].cpu().numpy().astype(np.complex128)
            out["nrmse_vs_fp64_sample_db"] = float(
                20 * np.log10(np.linalg.norm(s - sample[1]) / np.linalg.norm(sample[1])))
        return out

    rec.update(errors(img))

    def roofline_rows(kms, inf, leaf_ops, val_bytes, gemm="split_bf16"):
        """Per-kernel achieved rate against its bound, from the per-stage times."""
        rows = {}
        lms = kms.get("leaf_bp")
        if lms:
            a = inf["leaf_pairs"] * leaf_ops / (lms * 1e-3)
            rows["leaf_bp"] = {"bound": "alu", "ms": lms, "ops_per_pair": leaf_ops,
                               "pairs": inf["leaf_pairs"], "achieved": a / 1e12,
                               "peak": VALU_PEAK_OPS / 1e12, "unit": "Tops/s",
                               "frac": a / VALU_PEAK_OPS}
        rms = kms.get("rc_gemm")
        if rms:
            # the GEMM's float32 flops; the split-bfloat16 kernel (complex64
            # storage) executes six bf16 partial products for each, on bf16 MFMA
            fl = 2.0 * w.n_pos * (2 * w.n_f) * (2 * inf["n_range_bins"])
            if gemm == "split_bf16":
                rows["rc_gemm"] = {"bound": "mfma", "kernel": "split bf16 (6 partial products per f32 product)",
                                   "ms": rms, "flop": 6 * fl, "achieved": 6 * fl / (rms * 1e-3) / 1e12,
                                   "peak": MFMA_BF16_PEAK / 1e12, "unit": "TFLOP/s",
                                   "frac": 6 * fl / (rms * 1e-3) / MFMA_BF16_PEAK,
                                   "f32_flop_rate": fl / (rms * 1e-3) / 1e12}
            else:
                rows["rc_gemm"] = {"bound": "mfma", "kernel": "f32", "ms": rms, "flop": fl,
                                   "achieved": fl / (rms * 1e-3) / 1e12, "peak": MFMA_F32_PEAK / 1e12,
                                   "unit": "TFLOP/s", "frac": fl / (rms * 1e-3) / MFMA_F32_PEAK}
        # interpolation kernels: the merges gather through the vector L1 (16
        # column bases of 4 B, 64 taps, the 24-B record per pair), which bounds
        # them; the final stage reads its taps from LDS and is VALU-bound (the
        # algorithmic count)
        gb = 16 * 4 + 64 * val_bytes + 24
        mpairs = {}
        for name, t in kms.items():
            if name.startswith("merge_d") or name == "final":
                mpairs[name] = t
        for name, t in mpairs.items():
            pairs = inf["final_pairs"] if name == "final" else None
            if pairs is None:
                # pairs of the merge at depth d: that depth's points x children
                pairs = inf["merge_pairs_depth"][int(name[len("merge_d"):])]
            if not pairs:
                continue
            va = pairs * INTERP_OPS_PER_PAIR / (t * 1e-3)
            ga = pairs * gb / (t * 1e-3)
            if name == "final":
                rows[name] = {"bound": "alu", "ms": t, "pairs": pairs,
                              "ops_per_pair": INTERP_OPS_PER_PAIR, "achieved": va / 1e12,
                              "peak": VALU_PEAK_OPS / 1e12, "unit": "Tops/s",
                              "frac": va / VALU_PEAK_OPS}
            else:
                rows[name] = {"bound": "l1", "ms": t, "pairs": pairs,
                              "gather_bytes_per_pair": gb, "achieved": ga / 1e12,
                              "peak": L1_PEAK_BPS / 1e12, "unit": "TB/s",
                              "frac": ga / L1_PEAK_BPS, "ops_per_pair": INTERP_OPS_PER_PAIR,
                              "valu_frac": va / VALU_PEAK_OPS}
        return rows

    kern = roofline_rows(kernels_ms, info, LEAF_OPS_LINEAR, 8)
    lr = kern["leaf_bp"]
    # algorithmic bytes of the level-1 BP: profiles + leaf points (32 B) + antenna
    # offsets (16 B) in, subimages out (8 B per point)
    pts = info["level_points"][-1]
    rec["roofline"] = {"kernel": "leaf_bp", "bound": "alu", "achieved": lr["achieved"],
                       "peak": lr["peak"], "unit": "Tops/s", "frac": lr["frac"],
                       "traffic": measured_traffic("leaf_bp"),
                       "ops_per_pair": LEAF_OPS_LINEAR, "pairs_per_launch": info["leaf_pairs"],
                       "avg_launch_ms": lr["ms"],
                       "algorithmic_bytes": w.n_pos * info["n_range_bins"] * 8 + pts * 32
                       + w.n_pos * 16 + pts * 8}
    rec["kernels_roofline"] = kern

    log("parity mode (ES range kernel), half storage and the S = 3 voxel-root form")
    extra = {}
    pl_es = H.Plan(*args3, range_kernel="es", range_oversample=2.0, range_taps=7, **form)
    ms_es, k_es, img_es = timed(pl_es, ech, max(3, args.steps // 2), args.warmup)
    extra["hhffbp_es"] = {"value": vp / (ms_es * 1e-3), "ms": ms_es, "kernels_ms": k_es,
                          "mode": "ES U=2 W=7 (parity mode), same grids",
                          "leaf_bp_roofline": roofline_rows(k_es, info, LEAF_OPS_ES, 8).get("leaf_bp"),
                          **errors(img_es)}
    del pl_es, img_es
    for st in ("f16", "bf16"):
        pl_h = H.Plan(*args3, range_kernel="linear", range_oversample=BENCH_U, storage=st, **form)
        eh = H.Plan.pack_echoes(ech, st)
        ms_h, k_h, img_h = timed(pl_h, eh, max(3, args.steps // 2), args.warmup)
        extra[f"hhffbp_{st}"] = {
            "value": vp / (ms_h * 1e-3), "ms": ms_h, "kernels_ms": k_h,
            "mode": f"{st} storage of echoes, profiles and subimages, f32 arithmetic",
            "nrmse_vs_f32_storage": (torch.linalg.norm(img_h - img) / torch.linalg.norm(img)).item(),
            **errors(img_h)}
        del pl_h, eh, img_h
    # the fused range compression + level-1 BP (one kernel, profiles in LDS)
    pl_f = H.Plan(*args3, range_kernel="linear", range_oversample=BENCH_U, range_fused=True, **form)
    ms_f, k_f, img_f = timed(pl_f, ech, max(3, args.steps // 2), args.warmup)
    extra["hhffbp_fused"] = {
        "value": vp / (ms_f * 1e-3), "ms": ms_f, "kernels_ms": k_f,
        "mode": "range compression fused into the level-1 BP (range_fused), same plan",
        "nrmse_vs_two_kernel_form": (torch.linalg.norm(img_f - img) / torch.linalg.norm(img)).item(),
        **errors(img_f)}
    del pl_f, img_f
    # the same plan with uniform grids (leaf grids at the other grids' oversampling)
    alt = dict(form, oversample_leaf=None)
    pl_a = H.Plan(*args3, range_kernel="linear", range_oversample=BENCH_U, **alt)
    ms_a, k_a, img_a = timed(pl_a, ech, max(3, args.steps // 2), args.warmup)
    extra["hhffbp_uniform_grids"] = {"value": vp / (ms_a * 1e-3), "ms": ms_a, "kernels_ms": k_a,
                                     "mode": f"the same plan with every grid at {list(BL_GAMMA)} "
                                             f"(S={alt['stages']}, root grid {alt['root_grid']})",
                                     "work": {k: pl_a.info()[k] for k in ("leaf_pairs", "level_points")},
                                     **errors(img_a)}
    del pl_a, img_a
    # the same plan with the float32 MFMA range compression
    pl_g = H.Plan(*args3, range_kernel="linear", range_oversample=BENCH_U, range_gemm="f32", **form)
    ms_g, k_g, img_g = timed(pl_g, ech, max(3, args.steps // 2), args.warmup)
    extra["hhffbp_f32_gemm"] = {
        "value": vp / (ms_g * 1e-3), "ms": ms_g, "kernels_ms": k_g,
        "mode": "the same plan with the float32 MFMA range-compression GEMM",
        "rc_gemm_roofline": roofline_rows(k_g, info, LEAF_OPS_LINEAR, 8, gemm="f32").get("rc_gemm"),
        "nrmse_vs_split_gemm": (torch.linalg.norm(img_g - img) / torch.linalg.norm(img)).item(),
        **errors(img_g)}
    del pl_g, img_g
    torch.cuda.empty_cache()

    log("direct-BP baselines")
    candidates = {}
    for u in DIRECT_U:
        fast = H.Plan(*args3, mode="direct_rc", range_kernel="linear", range_oversample=u)
        dimg = fast.image(ech)
        torch.cuda.synchronize()
        nd = 2 if index == 2 else 3
        d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        d0.record(stream)
        for _ in range(nd):
            fast.image(ech, out=dimg)
        d1.record(stream)
        torch.cuda.synchronize()
        candidates[f"linear U={u:g}"] = (d0.elapsed_time(d1) / nd,
                                         (torch.linalg.norm(dimg - ref) / nref).item())
        del fast, dimg
    ok = {k: v for k, v in candidates.items() if 20 * np.log10(v[1]) <= -30.0}
    d_mode = min(ok, key=lambda k: ok[k][0])
    dms, d_nrmse = ok[d_mode]
    direct_vp = vp / (dms * 1e-3)
    ex_plan = H.Plan(*args3, mode="direct_exact")
    ex_img = ex_plan.image(ech)
    torch.cuda.synchronize()
    x0, x1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    x0.record(stream)
    ex_plan.image(ech, out=ex_img)
    x1.record(stream)
    torch.cuda.synchronize()
    ex_ms = x0.elapsed_time(x1)
    ex_err = errors(ex_img)
    del ex_img, ex_plan
    rec.update({
        "reference": "float32 direct BP, ES range kernel U=2 W=7 (<= 1e-5 of float64 eq. 4), "
                     "full grid" + ("; float64 eq. (4) on the stored stratified sample of "
                                    "22212 voxels" if index == 2 else ""),
        **extra,
        "direct_bp": {"value": direct_vp, "unit": "vp/s", "ms": dms, "mode": d_mode,
                      "nrmse_vs_es_direct_db": 20 * np.log10(d_nrmse),
                      "candidates": {k: {"ms": v[0], "nrmse_vs_es_direct_db": 20 * np.log10(v[1])}
                                     for k, v in candidates.items()}},
        "direct_exact": {"value": vp / (ex_ms * 1e-3), "unit": "vp/s", "ms": ex_ms,
                         "mode": f"eq. (4): Horner sum over the {w.n_f} frequencies per pair",
                         **ex_err},
        "speedup_vs_direct": value / direct_vp,
    })
    return rec


def valu_probe_report(args):
    """Issue rate of wave64 FP32 FMAs and transcendentals on the device
    (libhhffbp_probe.so, built with the package): what the nominal VALU peak of
    the rooflines comes to, and what a sine or square root costs."""
    import ctypes

    import torch

    from paper_2506_23568_amd import build_lib

    if not os.path.exists(build_lib.PROBE_LIB):
        raise RuntimeError("libhhffbp_probe.so is missing: run __graft_entry__.build()")
    L = ctypes.CDLL(build_lib.PROBE_LIB)
    L.hhffbp_probe_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_double)]
    L.hhffbp_probe_valu.restype = ctypes.c_int
    blocks, iters, reps = 256 * 8, 2048, 5
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    nominal = 256 * 4 * 2.4e9 / 4  # wave64 instructions per second at 4 cycles each
    names = ["4 fma", "4 sine", "3 fma + 1 sine (one chain)", "4 sqrt", "2 fma + 2 sine",
             "3 fma + 1 sine (independent chains)", "4 fma (two chains)",
             "level-1 BP mix: 20 fma + sqrt, rcp, sine, cosine"]
    rows = {}
    for mode, name in enumerate(names):
        r = ctypes.c_double(0.0)
        rc = L.hhffbp_probe_valu(mode, blocks, iters, reps, ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(st), ctypes.byref(r))
        if rc != 0:
            raise RuntimeError(f"probe mode {mode} failed: {rc}")
        rows[name] = {"wave_instr_per_s": r.value, "frac_of_nominal": r.value / nominal}
        log(f"{name}: {r.value:.3e} wave64 instructions/s = {r.value / nominal:.3f} of nominal")
    print(json.dumps({"metric": "wave64 VALU instructions per second", "unit": "instr/s",
                      "nominal": nominal, "blocks": blocks, "iters": iters, "reps": reps,
                      "modes": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-timed", action="store_true",
                    help="time the benchmarked form alone (no references, no other forms): "
                         "for kernel traces and counter runs")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="run one plain copy of this size first (HBM counter scale)")
    ap.add_argument("--af-range", choices=("es", "linear"), default="linear",
                    help="range kernel of the autofocus workload's images")
    ap.add_argument("--af-u", type=float, default=4.0,
                    help="autofocus workload: range oversampling of the linear range kernel")
    ap.add_argument("--af-stages", type=int, default=4,
                    help="autofocus workload: merge stages S")
    ap.add_argument("--af-root-grid", choices=("on", "off"), default="on",
                    help="autofocus workload: plans with a compressed root grid (the "
                         "last merge onto the full aperture's lattice, one resample to "
                         "the voxels)")
    ap.add_argument("--workload", choices=["large", "mid", "autofocus", "paper_sim", "valu_probe"],
                    default="large",
                    help="large: the imaging benchmark (default; the mid workload is "
                         "reported beside it); mid: the mid workload alone; autofocus: "
                         "the trajectory correction loop on the large scene; paper_sim: "
                         "the paper's simulation geometry with point-response metrics; "
                         "valu_probe: the device's FMA and transcendental issue rates")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the voxel "
              "grid would be split into slabs, one per GPU)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "autofocus":
        autofocus_report(args)
        return
    if args.workload == "paper_sim":
        paper_sim_report(args)
        return
    if args.workload == "valu_probe":
        valu_probe_report(args)
        return

    import torch

    if args.copy_mib > 0:
        copy_probe(torch, args.copy_mib)
    index = 2 if args.workload == "large" else 1
    rec = imaging_report(args, index)
    if index == 2 and not args.only_timed:
        log("the mid workload beside it")
        mid = imaging_report(args, 1)
        rec["mid"] = {k: mid[k] for k in ("value", "ms_per_step", "config", "kernels_ms",
                                          "kernels_roofline", "nrmse_vs_direct_db", "work",
                                          "direct_bp", "speedup_vs_direct")}
    cpu = None
    if not args.no_cpu_baseline and not args.only_timed:
        log("oracle CPU baseline")
        from workloads import make_config
        w = make_config(index, synth_device="cuda")
        cpu = oracle_cpu_baseline(w, index)
    rec["cpu_baseline"] = cpu
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
