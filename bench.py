"""Benchmark: cell-updates/s of the temporal-adaptive finite-volume Euler
path on one MI355X.

Workload (one step): the 64^3 hex grid graded 16x toward the origin, each
hex split into 6 tets (1,572,864 cells), second-order MUSCL (least squares +
Barth-Jespersen), exact Riemann flux with Newton on p* (tol 1e-12), up to 5
temporal levels, a spherical blast (rho = 1, u = 0, p = 10 within 0.2 of a
centre drawn from seed 0 in [0.3, 0.7]^3, p = 1 elsewhere), reflective
walls, advanced 32 dt_min units from the initial state (the state is
restored on the device before every step).  FP64 throughout.  Device memory
comes from PyTorch's caching allocator (tafv_set_allocator); the library
launches its own kernels on PyTorch's current stream.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

UNITS = 32
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per work item of each kernel class (each input and
# output moved once per item):
#   flux (per face): index 4, half-face ids 8, area vector 24 (12 in FP32),
#     levels 2, two reconstructed states 80 (40), read+write of two FP64
#     accumulators 160;
#   grad (per cell): index 4, own state 40, neighbour ids 16,
#     reconstruction coefficients 96 (48), 4 reconstructed face states
#     160 (80);
#   update (per cell): index 4, volume 8, state read+write 80, accumulator
#     read+write 80.
BYTES_PER_ITEM = {
    "fp64": {"flux": 278, "grad": 316, "update": 172},
    "fp32": {"flux": 226, "grad": 188, "update": 172},
}
# gather mode: the flux kernel reads the face's key and half-face ids (9
# bytes; launches over most of the faces walk them in face order, which
# carry most face solves; a launch over the level-sorted list reads a
# 16-byte record instead), the area vector, two reconstructed states and
# writes one flux (5 values in the flux precision); the cell kernel reads
# its index, its packed level word, 4 face ids, the active faces' fluxes
# (about 2 per cell), reads+writes the FP64 accumulator, and for ending steps
# the volume and state.
BYTES_PER_ITEM_GATHER = {
    "fp64": {"flux": 153, "grad": 316, "gather": 270},
    "fp32": {"flux": 81, "grad": 188, "gather": 230},
}
# the other forms (gather mode): the predictor/corrector form's corrector
# pass also reads the predictor flux (5 values in the flux precision) and its
# cell kernel also writes the corrected state to the interpolated-state array
# (40 bytes); a moving mesh's flux kernel also reads the face's volume rate
# (8) and its cell kernel about two volume rates (16) and the pending swept
# volume read + write (16).
BYTES_PER_ITEM_FORM = {
    "fp64": BYTES_PER_ITEM_GATHER["fp64"],
    "fp32": BYTES_PER_ITEM_GATHER["fp32"],
    "fp32_learned": BYTES_PER_ITEM_GATHER["fp32"],
    "time2_fp64": {"flux": 153, "flux_corrector": 193, "grad": 316, "gather": 310},
    "time2_fp32": {"flux": 81, "flux_corrector": 101, "grad": 188, "gather": 270},
    "moving_fp64": {"flux": 161, "grad": 316, "gather": 302},
}
# kernel of each timing class, by form (names of the counter records)
KERNEL_OF_CLASS = {"flux": "k_flux", "flux_corrector": "k_flux", "grad": "k_grad",
                   "gather": "k_gather", "update": "k_update", "grad_flux": "k_grad_flux"}
# Whole-mesh gradient launches that also compute the faces local to a chunk
# of 256 cells (k_grad_flux): per cell in range the gradient's bytes less
# the face values kept on chip (160 FP64, 80 FP32, times the share f of
# half-faces local to a chunk), per local face its entry of the chunk's list
# (8), its area vector (24; 12), the lower cell's packed level word (4) and
# its flux (40; 20).
GRAD_FLUX_BYTES = {"fp64": (316, 160, 76), "fp32": (188, 80, 44)}


def local_half_face_share(T, cfg):
    """Share of half-faces whose other side lies in the same chunk of 256
    cells of the mesh order (boundary half-faces included)."""
    nb = T.tafv_mesh_inspect(cfg["nodes"], cfg["tets"])["cell_neighbours"]
    i = np.arange(len(nb))[:, None]
    return float(((nb < 0) | (nb // 256 == i // 256)).mean())


def log(*a):
    print(*a, file=sys.stderr, flush=True)


CELL_ORDER = 1  # internal cell order of the single-mesh runs (set from --cell-order)
FUSE_FACES = 0  # chunk-local faces computed by the gradient launches (set from --fuse-faces)
PIPELINE_CHUNKS = 1  # pipelined whole-mesh subiterations (set from --pipeline-chunks)


def run_form(T, torch, cfg, precision, steps, warmup, scatter, mlp=None, stats=0, time_order=1,
             motion=None):
    stream = torch.cuda.current_stream()
    extra = dict(guess_stats=stats)
    if mlp is not None:
        extra = dict(guess=T.GUESS_MLP, guess_stats=stats, guess_gate=mlp["gate"],
                     guess_strength=mlp["strength"])
    s = T.Solver(device=0, hip_stream=stream.cuda_stream, max_levels=cfg["max_levels"],
                 order=cfg["order"], precision=precision, scatter=scatter, time_order=time_order,
                 cell_order=CELL_ORDER, fuse_faces=FUSE_FACES, pipeline_chunks=PIPELINE_CHUNKS,
                 allocator=T.torch_allocator(0, stream), **extra)
    s.upload(cfg["nodes"], cfg["tets"])
    if mlp is not None:
        T.tafv_mlp_set(s.ctx, mlp["theta"])
    s.init(cfg["prim"])
    if motion is not None:
        s.motion(motion)  # kept across the resets; each reset restores the volumes
    for _ in range(warmup):
        s.reset()
        T.tafv_advance_async(s.ctx, UNITS)
    torch.cuda.synchronize()
    st0 = s.stats()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        s.reset()
        T.tafv_advance_async(s.ctx, UNITS)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    st1 = s.stats()
    # the same steps again with HIP events around every kernel launch (on
    # the library's stream) for the per-kernel times; the events cost a few
    # per cent of the step, so the throughput above is taken without them
    T.tafv_profile_enable(s.ctx, True)
    T.tafv_profile_read(s.ctx)  # clear
    ev0.record(stream)
    for _ in range(steps):
        s.reset()
        T.tafv_advance_async(s.ctx, UNITS)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_prof = ev0.elapsed_time(ev1)
    prof = T.tafv_profile_read(s.ctx)
    T.tafv_profile_enable(s.ctx, False)
    updates = st1["cell_updates"] - st0["cell_updates"]
    faces = st1["face_solves"] - st0["face_solves"]
    newton = st1["newton_updates"] - st0["newton_updates"]
    cons, lev = s.read()
    s.close()
    hist = (np.array(st1["newton_hist"]) - np.array(st0["newton_hist"])).tolist()
    return dict(ms=ms, ms_prof=ms_prof, wall_s=wall, updates=updates, faces=faces, newton=newton,
                prof=prof, newton_hist=hist,
                stats=st1, cons=cons, levels=lev,
                gated=st1["guess_faces"] - st0["guess_faces"],
                gated_newton=st1["guess_newton_updates"] - st0["guess_newton_updates"],
                used=st1["guess_used"] - st0["guess_used"],
                evaluated=st1["guess_evaluated"] - st0["guess_evaluated"])


def train_guess(T, torch, I, n, train_seeds=(1, 2, 3, 4, 5), rows_per_seed=400000):
    """Learned p* guess: log face states from blasts with the training seeds
    (FP64 path, full run each), train on the GPU, choose the gate by the
    GPU's own Newton-update counters on a training seed.  Returns the
    parameters, the gate and the training figures."""
    stream = torch.cuda.current_stream()
    cfg = I.config_scale(n, train_seeds[0])
    s = T.Solver(device=0, hip_stream=stream.cuda_stream, max_levels=cfg["max_levels"],
                 order=cfg["order"], guess_stats=1, allocator=T.torch_allocator(0, stream))
    s.upload(cfg["nodes"], cfg["tets"])
    rows = []
    for seed in train_seeds:
        prim = I.blast_state(cfg["nodes"], cfg["tets"], centre=I.blast_centre(seed))
        s.init(prim)
        T.tafv_facelog_config(s.ctx, rows_per_seed, 0.75, seed)
        T.tafv_advance(s.ctx, UNITS)
        rows.append(T.tafv_facelog_read(s.ctx, rows_per_seed))
    rows = np.concatenate(rows)
    T.tafv_mlp_set(s.ctx, I.mlp_init(0))
    t0 = time.perf_counter()
    loss = T.tafv_mlp_train(s.ctx, rows[:, :6], rows[:, 6], epochs=20, batch=4096, lr=2e-3,
                            seed=11)
    train_s = time.perf_counter() - t0
    theta = T.tafv_mlp_get(s.ctx)
    # strength pre-gate: the network is worth evaluating where the
    # two-rarefaction value is off by more than 2%; take the jump strength
    # |u_R - u_L|/a_m + |p_L - p_R|/p_m that keeps 90% of those training rows
    strength = 2.0 * (np.abs(rows[:, 1]) + np.abs(rows[:, 2]))
    useful = np.abs(rows[:, 6]) > 0.02
    s0 = float(np.quantile(strength[useful], 0.1)) if useful.any() else float("inf")
    # gate: mean Newton updates per inexact-TR face on the first training seed
    prim = I.blast_state(cfg["nodes"], cfg["tets"], centre=I.blast_centre(train_seeds[0]))
    T.tafv_facelog_config(s.ctx, 0, 0.0, 0)
    per_gate = {}
    for gate in (None, 0.0, 0.01, 0.03, 0.1):
        if gate is None:
            T.tafv_guess_config(s.ctx, T.GUESS_TR, 0.0, 1)
        else:
            T.tafv_guess_config(s.ctx, T.GUESS_MLP, gate, 1, strength=s0)
        s.init(prim)
        st = T.tafv_advance(s.ctx, UNITS)
        per_gate["tr" if gate is None else gate] = st["guess_newton_updates"] / max(st["guess_faces"], 1)
    s.close()
    best = min((g for g in per_gate if g != "tr"), key=lambda g: per_gate[g])
    return dict(theta=theta, gate=best, strength=s0, rows=int(len(rows)),
                rows_useful=int(useful.sum()), train_s=round(train_s, 3),
                loss_first=float(loss[0]), loss_last=float(loss[-1]),
                newton_per_inexact_face={str(k): round(v, 4) for k, v in per_gate.items()})


BATCH_UNITS = 16


def run_batch(T, torch, cases, steps, warmup, precision, mlp=None, graph=1):
    """The batched form: every mesh of `cases` in one context (params.batch),
    HIP graphs and the autotuner on; each step restores all initial states
    on the device and advances 16 dt_min units."""
    stream = torch.cuda.current_stream()
    extra = {}
    if mlp is not None:
        extra = dict(guess=T.GUESS_MLP, guess_gate=mlp["gate"], guess_strength=mlp["strength"])
    t0 = time.perf_counter()
    s = T.Solver(device=0, hip_stream=stream.cuda_stream, batch=1, order=2,
                 precision=precision, allocator=T.torch_allocator(0, stream), **extra)
    for c in cases:
        s.upload(c["nodes"], c["tets"], max_levels=c["max_levels"])
    T.tafv_batch_config(s.ctx, graph, 1, None)
    if mlp is not None:
        T.tafv_mlp_set(s.ctx, mlp["theta"])
    for k, c in enumerate(cases):
        s.init(c["prim"], mesh_id=k)
    setup_s = time.perf_counter() - t0
    for _ in range(warmup):
        T.tafv_state_reset(s.ctx, -1)
        T.tafv_advance(s.ctx, BATCH_UNITS)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    tot = dict(cell_updates=0, face_solves=0, newton_updates=0, guess_faces=0,
               guess_newton_updates=0, guess_used=0, guess_evaluated=0)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        T.tafv_state_reset(s.ctx, -1)
        st = T.tafv_advance(s.ctx, BATCH_UNITS)
        for k in tot:
            tot[k] += st[k]
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    info = T.tafv_batch_info(s.ctx)
    cons = [s.read(k)[0] for k in range(len(cases))]
    s.close()
    return dict(ms=ms, setup_s=setup_s, info=info, cons=cons, **tot)


def run_group(T, torch, cases, steps, warmup, precision, mlp=None, workers=8, nstreams=8):
    """The batched workload run the task-based way: one single-mesh context
    per mesh, contexts spread over `nstreams` streams, all advanced together
    by tafv_advance_group with `workers` host threads (each mesh's
    subiterations are chained on its stream; no mesh waits for another at a
    subiteration boundary).  Timed on the host clock between two device
    synchronisations (several streams)."""
    extra = {}
    if mlp is not None:
        extra = dict(guess=T.GUESS_MLP, guess_gate=mlp["gate"], guess_strength=mlp["strength"])
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    t0 = time.perf_counter()
    ss = []
    for k, c in enumerate(cases):
        st = streams[k % nstreams]
        s = T.Solver(device=0, hip_stream=st.cuda_stream, order=2, precision=precision,
                     max_levels=c["max_levels"], allocator=T.torch_allocator(0, st), **extra)
        s.upload(c["nodes"], c["tets"])
        if mlp is not None:
            T.tafv_mlp_set(s.ctx, mlp["theta"])
        s.init(c["prim"])
        ss.append(s)
    setup_s = time.perf_counter() - t0
    ctxs = [s.ctx for s in ss]

    def step():
        for s in ss:
            T.tafv_state_reset(s.ctx, 0)
        T.tafv_advance_group(ctxs, BATCH_UNITS, workers, stats=False)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    u0 = sum(s.stats()["cell_updates"] for s in ss)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    u1 = sum(s.stats()["cell_updates"] for s in ss)
    cons = [s.read()[0] for s in ss]
    for s in ss:
        s.close()
    return dict(ms=wall * 1e3, setup_s=setup_s, cell_updates=u1 - u0, cons=cons)


def batch_l1(cases, ref, got):
    worst = 0.0
    for c, a, b in zip(cases, got, ref):
        p = c["nodes"][c["tets"]]
        vol = np.einsum("ij,ij->i", p[:, 1] - p[:, 0],
                        np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0])) / 6.0
        for k in (0, 4):
            worst = max(worst, float((vol * np.abs(a[:, k] - b[:, k])).sum()
                                     / (vol * np.abs(b[:, k])).sum()))
    return worst


def l1_errors(cfg, ref, got):
    p = cfg["nodes"][cfg["tets"]]
    vol = np.einsum("ij,ij->i", p[:, 1] - p[:, 0], np.cross(p[:, 2] - p[:, 0], p[:, 3] - p[:, 0])) / 6.0
    e = [float((vol * np.abs(got[:, k] - ref[:, k])).sum() / (vol * np.abs(ref[:, k])).sum())
         for k in (0, 4)]
    return e


def measured_traffic(kernel, form):
    """HBM bytes per launch of `kernel` in `form` from the committed counter
    record (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when
    there is no record or the library sources changed after it was taken."""
    from paper_1704_01144_amd import profile_summary as PS
    path = os.path.join(ROOT, "profiles", f"{kernel}_graded64_blast_{form}_counters.txt")
    if not os.path.exists(path):
        return None, "no counter record"
    rec = PS.read_record(path)
    if rec.get("sources_sha256") != PS.source_digest():
        return None, "sources changed since the counters were taken"
    return int(float(rec["traffic_bytes_per_launch"])), os.path.relpath(path, ROOT)


def roofline(prof, bytes_per_item, form, class_bytes=None):
    """Roofline entry of the longest kernel class of a run with a known
    algorithmic byte count: per item (bytes_per_item), or in total for the
    run (class_bytes)."""
    class_bytes = class_bytes or {}
    known = set(bytes_per_item) | set(class_bytes)
    dom = max((k for k in prof if k in known and prof[k]["items"] > 0),
              key=lambda k: prof[k]["ms"])
    p = prof[dom]
    total = class_bytes[dom] if dom in class_bytes else bytes_per_item[dom] * p["items"]
    achieved = total / (p["ms"] * 1e-3) / 1e9
    name = KERNEL_OF_CLASS[dom] + ("_corrector" if dom == "flux_corrector" else "")
    traffic, src = measured_traffic(name, form)
    launches = max(p["launches"], 1)
    return dom, {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                 "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                 "traffic_unit": "HBM bytes per launch", "traffic_source": src,
                 "kernel": name, "timing_class": dom,
                 "avg_launch_us": round(1e3 * p["ms"] / launches, 2),
                 "bytes_per_item": round(total / max(p["items"], 1), 1), "items": p["items"],
                 "launches": p["launches"],
                 "algorithmic_bytes_per_launch": int(total / launches)}


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Read + write GB/s of a plain device-to-device copy of nbytes, timed
    with events: the practical ceiling the kernels' traffic compares to."""
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(reps):
        y.copy_(x)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def copy_probe():
    """A plain device-to-device copy of 1 GiB, three times: the known-size
    kernel that the FETCH_SIZE / WRITE_SIZE counters are scaled by."""
    import torch
    n = 2 ** 27
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    log(f"copied {n * 8} bytes three times")


def host_cpu():
    """CPU model and logical core count of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(cfg, units=24, variant="seq", repeats=1):
    """The oracle on the first `units` subiterations of the same workload,
    `repeats` times from the initial state: variant "seq" is the sequential
    parity reference (one thread; 24 units, three full iterations at
    theta = 3, about 15 s), "omp" the same source built with OpenMP (same
    bits, per-cell and per-face loops on all the host threads that
    OMP_NUM_THREADS allows)."""
    from oracle import core as orc
    orc.select(variant)
    try:
        m = orc.Mesh(cfg["nodes"], cfg["tets"])
        prm = orc.params(max_levels=cfg["max_levels"], order=cfg["order"])
        threads = orc.threads()
        dt, updates = 0.0, 0
        for _ in range(repeats):
            o = orc.State(m, cfg["prim"], prm)
            t0 = time.perf_counter()
            o.advance(units)
            dt += time.perf_counter() - t0
            updates += o.stats()["cell_updates"]
    finally:
        orc.select("seq")
    model, ncpu = host_cpu()
    what = f"first {units} of {UNITS} dt_min units" if units < UNITS else f"{UNITS} dt_min units"
    return {"value": round(updates / dt, 1), "unit": "cell-updates/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{what}{f', {repeats} times' if repeats > 1 else ''} (cell updates "
                      f"{updates}, {dt:.1f} s) on the same 1,572,864-cell mesh and state, FP64, "
                      f"{threads} thread{'s' if threads > 1 else ''}"
                      + (" (OpenMP build of the same source, bit-identical)" if threads > 1 else ""),
            "host_cpu": model, "host_logical_cpus": ncpu}


FORMS = ("fp64", "fp32_flux", "fp32_learned", "time_order_2_fp64", "time_order_2_fp32_flux",
         "moving_mesh_fp64", "batched")


def with_roofline(entry, run, bpi, form, copy_gbs, f_loc=None):
    """Adds the roofline of the run's longest kernel (algorithmic bytes per
    launch over its average launch time, from HIP events on the library's
    stream), its share of a plain copy's bandwidth and the kernel times.
    f_loc: share of half-faces local to a chunk, for the fused launches."""
    extra = {}
    gf = run["prof"].get("grad_flux")
    if gf and gf["items"] > 0 and f_loc is not None:
        cell, wf, face = GRAD_FLUX_BYTES["fp32" if "fp32" in form else "fp64"]
        local_faces = run["faces"] - run["prof"].get("flux", {}).get("items", 0)
        extra["grad_flux"] = gf["items"] * (cell - wf * f_loc) + local_faces * face
        entry["faces_computed_in_gradient_launches"] = round(local_faces / max(run["faces"], 1), 4)
        entry["half_faces_local_to_a_chunk"] = round(f_loc, 4)
    _, roof = roofline(run["prof"], bpi, form, extra)
    if copy_gbs:
        roof["copy_gbs_measured"] = round(copy_gbs, 1)
        roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)
        if roof["traffic"] is not None:
            tgbs = roof["traffic"] / (roof["avg_launch_us"] * 1e-6) / 1e9
            roof["traffic_gbs"] = round(tgbs, 1)
            roof["traffic_frac_of_copy"] = round(tgbs / copy_gbs, 4)
    entry["roofline"] = roof
    entry["kernels_ms"] = {k: round(v["ms"], 3) for k, v in run["prof"].items()}
    return entry


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=64, help="hexes per axis")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--scatter", type=int, default=1, help="0 colour, 1 gather")
    ap.add_argument("--no-batch", action="store_true", help="skip the 128-mesh batched form")
    ap.add_argument("--no-time2", action="store_true",
                    help="skip the predictor/corrector form (second order in time)")
    ap.add_argument("--no-moving", action="store_true", help="skip the moving-mesh form")
    ap.add_argument("--only", choices=FORMS,
                    help="run this form alone (for profiling); prints its entry as the JSON line")
    ap.add_argument("--fuse-faces", type=int, default=0, choices=(0, 1),
                    help="1: whole-mesh gradient launches also compute the faces local to a "
                         "256-cell chunk; 0: every face through the flux kernel")
    ap.add_argument("--pipeline-chunks", type=int, default=1,
                    help="K > 1: whole-mesh subiterations as a pipeline over K chunks")
    ap.add_argument("--cell-order", type=int, default=1, choices=(0, 1),
                    help="internal cell order of the single-mesh runs: 0 the mesh's own, "
                         "1 Morton order of the centroids (the default; results are returned "
                         "in the mesh's order either way)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched form, FP64 and FP32 with the two-rarefaction start")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the 1 GiB copy used to scale the traffic counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is not implemented)", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        copy_probe()
        return
    global CELL_ORDER, FUSE_FACES, PIPELINE_CHUNKS
    CELL_ORDER = args.cell_order
    FUSE_FACES = args.fuse_faces
    PIPELINE_CHUNKS = args.pipeline_chunks

    import torch

    from paper_1704_01144_amd import inputs as I
    from paper_1704_01144_amd import tafv as T

    torch.cuda.set_device(0)
    if args.batch_only:
        cases = I.config_batch(128)
        for prec, name in ((T.FP64, "fp64"), (T.FP32_FLUX, "fp32")):
            r = run_batch(T, torch, cases, args.steps, args.warmup, prec)
            v = r["cell_updates"] / (r["ms"] * 1e-3)
            log(f"batched {name}: {v / 1e9:.3f} G cell-updates/s, {r['ms'] / args.steps:.2f} ms "
                f"per step, launch {r['info']}")
        return
    want = (lambda f: f == args.only) if args.only else (lambda f: True)
    if args.only:  # a single form: no reference run, baseline or copy timing
        args.no_cpu_baseline = True
    cfg = I.config_scale(args.n, 0)
    log(f"workload: {len(cfg['tets'])} cells, order {cfg['order']}, L {cfg['max_levels']}, "
        f"{UNITS} units, steps {args.steps}, warmup {args.warmup}")
    bpi = BYTES_PER_ITEM_GATHER if args.scatter == 1 else BYTES_PER_ITEM
    copy_gbs = None if args.only else copy_bandwidth(torch)
    f_loc = local_half_face_share(T, cfg)
    out = {}
    forms = {}
    r64 = None
    if want("fp64") or not args.only:
        r64 = run_form(T, torch, cfg, T.FP64, args.steps, args.warmup, args.scatter)
        value = r64["updates"] / (r64["ms"] * 1e-3)
        log(f"fp64: {r64['ms']:.2f} ms for {args.steps} steps, {value / 1e9:.3f} G cell-updates/s")
        head = with_roofline({}, r64, bpi["fp64"], "fp64", copy_gbs, f_loc)
        roof = head["roofline"]
        log(f"dominant kernel {roof['kernel']} at {roof['achieved']:.0f} GB/s algorithmic "
            f"({roof['frac']:.3f} of 8 TB/s)" +
            (f"; copy {copy_gbs:.0f} GB/s read+write" if copy_gbs else ""))
        out = {
            "metric": "cell-updates/s, 1.57M-tet graded mesh: FP64 plain vs FP32+learned @ L1 err",
            "value": round(value, 1),
            "unit": "cell-updates/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": round(r64["ms"] / args.steps, 4),
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"graded blast, {args.n}^3 hexes x 6 tets "
                                   f"({len(cfg['tets'])} cells), grading 16, MUSCL-LSQ + "
                                   f"Barth-Jespersen, exact Riemann (Newton tol 1e-12), <= 5 "
                                   f"levels, {UNITS} dt_min units, walls, seed 0",
                       "cells": len(cfg["tets"]), "units": UNITS,
                       "internal_cell_order": ("morton" if CELL_ORDER else "mesh"),
                       "cell_updates_per_step": r64["updates"] // args.steps,
                       "face_solves_per_step": r64["faces"] // args.steps,
                       "newton_updates_per_face": round(r64["newton"] / max(r64["faces"], 1), 3),
                       "levels_t0": r64["stats"]["cells_per_level"][:5]},
            "roofline": roof,
            "kernels_ms": head["kernels_ms"],
            **{k: head[k] for k in ("faces_computed_in_gradient_launches",
                                    "half_faces_local_to_a_chunk") if k in head},
            "profiled_pass_ms_per_step": round(r64["ms_prof"] / args.steps, 4),
        }

    def l1_vs_fp64(entry, run, ref=None):
        ref = ref if ref is not None else r64
        if ref is not None:
            entry["l1_rho"], entry["l1_E"] = l1_errors(cfg, ref["cons"], run["cons"])

    def rate(run):
        return run["updates"] / (run["ms"] * 1e-3)

    if not args.no_fp32 and want("fp32_flux"):
        r32 = run_form(T, torch, cfg, T.FP32_FLUX, args.steps, args.warmup, args.scatter)
        v32 = rate(r32)
        e = {"value": round(v32, 1), "ms_per_step": round(r32["ms"] / args.steps, 4)}
        if r64 is not None:
            e["speedup_vs_fp64"] = round(v32 / out["value"], 3)
            e["l1_reference"] = "FP64 GPU result of the same run (equal to the oracle within 1e-12)"
        l1_vs_fp64(e, r32)
        forms["fp32_flux"] = with_roofline(e, r32, bpi["fp32"], "fp32", copy_gbs, f_loc)
        log(f"fp32 flux: {v32 / 1e9:.3f} G/s, L1 rho {e.get('l1_rho', float('nan')):.2e}, "
            f"L1 E {e.get('l1_E', float('nan')):.2e}")
    g = None
    need_net = want("fp32_learned") or (want("batched") and not args.no_batch)
    if not args.no_fp32 and not args.no_learned and args.scatter == 1 and need_net:
        log("learned guess: logging seeds 1-5, training, gate choice ...")
        g = train_guess(T, torch, I, args.n)
    if g is not None and want("fp32_learned"):
        rl = run_form(T, torch, cfg, T.FP32_FLUX, args.steps, args.warmup, args.scatter, mlp=g)
        # the Newton counts on the faces where two-rarefaction is inexact
        # come from a run with statistics (they cost a little time)
        rs = run_form(T, torch, cfg, T.FP32_FLUX, 1, 0, args.scatter, mlp=g, stats=1)
        rs_tr = run_form(T, torch, cfg, T.FP32_FLUX, 1, 0, args.scatter, stats=1)
        vl = rate(rl)
        e = {"value": round(vl, 1), "ms_per_step": round(rl["ms"] / args.steps, 4)}
        if r64 is not None:
            e["speedup_vs_fp64"] = round(vl / out["value"], 3)
        if "fp32_flux" in forms:
            e["speedup_vs_fp32_flux"] = round(vl / forms["fp32_flux"]["value"], 4)
        l1_vs_fp64(e, rl)
        e.update({
            "gate": g["gate"], "train_rows": g["rows"], "train_seconds": g["train_s"],
            "train_loss_first_last": [g["loss_first"], g["loss_last"]],
            "newton_per_inexact_tr_face_by_gate": g["newton_per_inexact_face"],
            "strength_pregate": round(g["strength"], 5), "train_rows_tr_off_2pct": g["rows_useful"],
            "eval_newton_per_inexact_face": round(rs["gated_newton"] / max(rs["gated"], 1), 4),
            "eval_faces_network_evaluated_per_step": rs["evaluated"],
            "eval_faces_started_by_network_per_step": rs["used"],
            "newton_per_face_all": round(rs["newton"] / max(rs["faces"], 1), 4),
            # face solves of one step by category (rarefactions, one shock,
            # two shocks) and Newton updates (1..7, 8 or more)
            "newton_histogram_by_category": {"two_rarefaction_start": rs_tr["newton_hist"],
                                             "learned_start": rs["newton_hist"]}})
        forms["fp32_learned"] = with_roofline(e, rl, BYTES_PER_ITEM_FORM["fp32_learned"],
                                              "fp32_learned", copy_gbs)
        log(f"fp32 + learned: {vl / 1e9:.3f} G/s, gate {g['gate']}, "
            f"per-gate updates {g['newton_per_inexact_face']}")
    if not args.no_time2 and args.scatter == 1:
        rt64 = None
        for prec, name, tag in ((T.FP64, "fp64", "time2_fp64"),
                                (T.FP32_FLUX, "fp32_flux", "time2_fp32")):
            if prec == T.FP32_FLUX and args.no_fp32:
                continue
            if not want(f"time_order_2_{name}"):
                continue
            rt = run_form(T, torch, cfg, prec, args.steps, args.warmup, args.scatter, time_order=2)
            vt = rate(rt)
            e = {"value": round(vt, 1), "ms_per_step": round(rt["ms"] / args.steps, 4),
                 "cell_updates_per_step": rt["updates"] // args.steps,
                 "face_solves_per_step": rt["faces"] // args.steps}
            if r64 is not None:
                e["cost_vs_time_order_1"] = round(rt["ms"] / r64["ms"], 3)
            if prec == T.FP64:
                rt64 = rt
            elif rt64 is not None:
                l1_vs_fp64(e, rt, rt64)
            forms[f"time_order_2_{name}"] = with_roofline(e, rt, BYTES_PER_ITEM_FORM[tag], tag,
                                                          copy_gbs)
            log(f"time order 2, {name}: {vt / 1e9:.3f} G cell-updates/s, "
                f"{rt['ms'] / args.steps:.2f} ms per step")
    if not args.no_moving and args.scatter == 1 and want("moving_mesh_fp64"):
        vel = I.motion_field(cfg["nodes"], 0.05, seed=0)
        rm = run_form(T, torch, cfg, T.FP64, args.steps, args.warmup, args.scatter, motion=vel)
        vm = rate(rm)
        e = {"value": round(vm, 1), "ms_per_step": round(rm["ms"] / args.steps, 4),
             "motion": "inputs.motion_field(nodes, 0.05, seed=0): node velocities, faces move "
                       "with their nodes, volumes by the geometric conservation law",
             "cell_updates_per_step": rm["updates"] // args.steps}
        if r64 is not None:
            e["cost_vs_fixed_mesh"] = round(rm["ms"] / r64["ms"], 3)
        forms["moving_mesh_fp64"] = with_roofline(e, rm, BYTES_PER_ITEM_FORM["moving_fp64"],
                                                  "moving_fp64", copy_gbs)
        log(f"moving mesh, fp64: {vm / 1e9:.3f} G cell-updates/s, "
            f"{rm['ms'] / args.steps:.2f} ms per step")
    if (not args.no_batch and not args.no_fp32 and not args.no_learned and args.scatter == 1
            and g is not None and want("batched")):
        cases = I.config_batch(128)
        ncell = sum(len(c["tets"]) for c in cases)
        log(f"batched form: {len(cases)} meshes, {ncell} cells, {BATCH_UNITS} units ...")
        b64 = run_batch(T, torch, cases, args.steps, args.warmup, T.FP64)
        bl = run_batch(T, torch, cases, args.steps, args.warmup, T.FP32_FLUX, mlp=g)
        v64 = b64["cell_updates"] / (b64["ms"] * 1e-3)
        vl = bl["cell_updates"] / (bl["ms"] * 1e-3)
        forms["batched"] = {
            "workload": f"{len(cases)} graded tet meshes (5k-400k cells log-uniform, grading "
                        f"2-32, level cap 1-6, blast per mesh from seeds 1000-1127), "
                        f"{ncell} cells, {BATCH_UNITS} dt_min units per step",
            "cells": ncell,
            "fp32_learned": {"value": round(vl, 1), "ms_per_step": round(bl["ms"] / args.steps, 4),
                             "cell_updates_per_step": bl["cell_updates"] // args.steps,
                             "face_solves_per_step": bl["face_solves"] // args.steps,
                             "faces_network_evaluated_per_step": bl["guess_evaluated"] // args.steps,
                             "faces_started_by_network_per_step": bl["guess_used"] // args.steps,
                             "l1_max_over_meshes_rho_E": batch_l1(cases, b64["cons"], bl["cons"]),
                             "launch": bl["info"], "setup_s": round(bl["setup_s"], 1)},
            "fp64": {"value": round(v64, 1), "ms_per_step": round(b64["ms"] / args.steps, 4),
                     "cell_updates_per_step": b64["cell_updates"] // args.steps,
                     "launch": b64["info"], "setup_s": round(b64["setup_s"], 1)},
        }
        log(f"batched: fp64 {v64 / 1e9:.3f} G/s, fp32 + learned {vl / 1e9:.3f} G/s")
        # the same workload advanced task-wise: a context per mesh on 8
        # streams, 8 host workers (tafv_advance_group)
        grp = {}
        for name, prec, net, ref in (("fp64", T.FP64, None, b64), ("fp32_learned", T.FP32_FLUX, g, bl)):
            rg = run_group(T, torch, cases, args.steps, args.warmup, prec, mlp=net)
            vg = rg["cell_updates"] / (rg["ms"] * 1e-3)
            vb = ref["cell_updates"] / (ref["ms"] * 1e-3)
            grp[name] = {"value": round(vg, 1), "ms_per_step": round(rg["ms"] / args.steps, 4),
                         "cell_updates_per_step": rg["cell_updates"] // args.steps,
                         "vs_batched": round(vg / vb, 4),
                         "max_abs_diff_vs_batched": float(max(np.abs(a - b).max() for a, b in
                                                              zip(rg["cons"], ref["cons"]))),
                         "setup_s": round(rg["setup_s"], 1)}
            log(f"task group {name}: {vg / 1e9:.3f} G/s ({vg / vb:.3f} of the batched form)")
        forms["batched"]["task_group"] = {
            "how": "one single-mesh context per mesh on 8 streams, advanced together by "
                   "tafv_advance_group with 8 host workers (host clock, device synchronised)",
            **grp}
    if args.only:
        entry = out if args.only == "fp64" else forms.get(args.only, {})
        print(json.dumps({"form": args.only, **entry}), flush=True)
        return
    if forms:
        out["forms"] = forms
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle, 1 thread ...")
        out["cpu_baseline"] = cpu_baseline(cfg)
        log(f"cpu baseline: {out['cpu_baseline']['value']:.0f} cell-updates/s")
        log("cpu baseline: oracle, OpenMP build on the host threads ...")
        out["cpu_baseline_all_cores"] = cpu_baseline(cfg, UNITS, "omp", repeats=6)
        cb = out["cpu_baseline_all_cores"]
        log(f"cpu baseline, {cb['cores']} threads: {cb['value']:.0f} cell-updates/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
