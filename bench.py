"""Benchmark of the sliding-mesh mortar operator on one MI355X.

Workload (default): plane sliding interface, N = 5 (6x6 Gauss points per face),
128 x 64 face pairs, compressible Navier-Stokes (5 states + 3x5 lifted gradients per
point), Roe + Harten-Hyman + BR1 viscous flux, mu = 1e-4, displacement 0.0137 l_par per
stage (constant sliding speed; crosses whole faces every ~73 stages).  One step = one
Runge-Kutta stage of the operator: displacement update (split, index map on crossings,
FP64 projection-matrix assembly) + the fused mortar flux + the FP64 conservation residual
sums of the stage's fluxes (on the device, no synchronization).  Inputs are resident in HBM;
input/output sets are rotated (> 1 GB) so the 256 MB Infinity Cache cannot hold them.

Prints one JSON line: headline value = FP32 mortar points/s; the plain FP64 run of the
same workload is reported beside it, with HIP-event kernel timings, the HBM roofline of
the fused kernel and the FP64 CPU oracle timed on this host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=300)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--config", type=int, default=4,
                   help="workload: 4 = the turbine-like batch of three interfaces (default), "
                        "2 = plane N=5, 3 = annulus, 5 = plane N=9 Euler, 6/7 = cylinder/cone, 1 = tiny")
    p.add_argument("--no-fp64", action="store_true")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-stages", type=int, default=0,
                   help="oracle stages of the CPU baseline (0: about 15 s of work)")
    p.add_argument("--rotate-bytes", type=float, default=1.2e9)
    p.add_argument("--graph", action="store_true",
                   help="replay a captured HIP graph per stage (the default for batches)")
    p.add_argument("--eager", action="store_true",
                   help="eager launches per stage, also for batches")
    p.add_argument("--no-autotune", action="store_true",
                   help="launch with the library defaults instead of autotuned launches")
    p.add_argument("--tune-cache", default=None,
                   help="JSON file of earlier autotuner choices (read, and written on a miss)")
    p.add_argument("--precision", choices=("fp32", "bf16", "fp16"), default="fp32",
                   help="headline leg: FP32, or FP32 data with bf16 / fp16 projection GEMMs")
    p.add_argument("--no-lifting", action="store_true",
                   help="skip the BR1 lifting leg (config.lifting)")
    p.add_argument("--tuning", default=None,
                   help="VARIANT,TILE,GRID: launch the headline leg with this tuning instead of "
                        "autotuning it; TILE is one length for every interface or one per "
                        "interface separated by '/'")
    p.add_argument("--copy-calibration", type=float, default=0.0,
                   help="only run a plain device copy of this many MB (counter calibration)")
    p.add_argument("--stream-reference", type=float, default=0.0,
                   help="only time torch's device copy, read-only sum and fill of an FP32 "
                        "array of this many GiB (the rates plain streams reach on this GPU)")
    return p.parse_args()


def copy_calibration(mb):
    """A plain copy of known size: its FETCH_SIZE/WRITE_SIZE counters scale the counter
    readings of the mortar kernel to bytes."""
    import torch
    n = int(mb * 1e6) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))


def stream_rates(gib, legs=("copy", "sum", "fill"), reps=20):
    """HBM rates (GB/s) of plain streams over an FP32 array of `gib` GiB, each the
    average of `reps` back-to-back launches between two events: a device copy (bytes
    read plus written), a read-only sum, a fill (bytes written)."""
    import torch
    n = int(gib * (1 << 30)) // 4
    x = torch.rand(n, device="cuda")
    y = torch.empty_like(x)
    s = torch.empty((), device="cuda")
    table = {"copy": (lambda: y.copy_(x), 8 * n),
             "sum": (lambda: torch.sum(x, 0, out=s), 4 * n),
             "fill": (lambda: y.fill_(2.0), 4 * n)}
    out = {}
    for name in legs:
        fn, nbytes = table[name]
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3 / reps
        out[name + "_GBs"] = nbytes / sec / 1e9
    del x, y, s
    torch.cuda.empty_cache()
    return out


def stream_reference(gib, reps=20):
    """Context for the roofline fraction, which is always taken against the published
    peak: the rates plain streams reach on this GPU."""
    out = {"array_bytes": 4 * (int(gib * (1 << 30)) // 4), "reps": reps}
    out.update(stream_rates(gib, reps=reps))
    print(json.dumps(out))


TRAFFIC_PROFILES = {2: "profiles/k_mortar_flux_ns_n5_plane128x64_traffic.md",
                    3: "profiles/k_mortar_flux_rd_annulus_n7_512x64.md",
                    4: "profiles/k_mortar_flux_rd_batch_turbine_c4_traffic.md",
                    5: "profiles/k_mortar_flux_rd_euler_plane_n9_256x256.md"}


def sources_sha256(names):
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2008_04356_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(config, precision, tuning):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter
    summary: its lines "launch variant=V tile_len=T[,T..] grid=G traffic=BYTES
    sources=a,b,.. sha256=HEX" give the measured traffic of one launch each (one tile
    length per interface of the launch).  None when there is none for
    this workload and launch, or the kernel sources have changed since the counters were
    taken."""
    rel = TRAFFIC_PROFILES.get(config)
    if rel is None or precision != "fp32" or not tuning:
        return None
    path = os.path.join(ROOT, rel)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if not line.startswith("launch "):
            continue
        try:
            kv = dict(x.split("=", 1) for x in line.split()[1:])
            if any(int(kv[k]) != tuning[0][k] for k in ("variant", "grid")):
                continue
            # one tile length per interface of the launch (comma-separated for a batch)
            if [int(t) for t in kv["tile_len"].split(",")] != [t["tile_len"] for t in tuning]:
                continue
            if sources_sha256(kv["sources"].split(",")) != kv["sha256"]:
                return None
            return int(kv["traffic"])
        except (KeyError, ValueError, OSError):
            return None
    return None


# kernel (symbol name) of each launch variant
KERNEL_OF_VARIANT = {0: "k_mortar_flux (VALU projections, 48 KB LDS)", 1: "k_mortar_flux_mfma",
                     2: "k_mortar_flux_rd", 3: "k_mortar_flux (VALU projections, 72 KB LDS)",
                     4: "k_mortar_flux_hyb"}


def algorithmic_bytes(spec):
    """Bytes one flux launch must move: every input value read once and every output
    value written once (per mortar point: (V_in + 5) values, V_in = 20 for NS, 5 Euler),
    plus the static metrics if they are per point."""
    b = 8 if spec.precision == 0 else 4
    per_face_point = (spec.n_in_vars * 2 + 5 * 2) * b   # both sides' inputs and outputs
    total = per_face_point * spec.P * spec.n_pairs
    if spec.metrics is not None:
        total += 4 * b * spec.P * spec.n_pairs
    return total


def lifting_bytes(spec):
    """Bytes one lifting launch must move: both sides' states in (plus the static metrics
    if they are per point) and both sides' 15 output values per face point out."""
    b = 8 if spec.precision == 0 else 4
    total = (5 * 2 + 15 * 2) * b * spec.P * spec.n_pairs
    if spec.metrics is not None:
        total += 4 * b * spec.P * spec.n_pairs
    return total


def run_leg(M, W, specs, disp, steps, warmup, rotate_bytes, graph=False, plain=False, tune=True,
            tune_cache=None, fixed=None, measure_lifting=False):
    """Times one precision of a workload.  plain: one handle (one launch) per interface
    instead of the batched persistent launch; graph: each stage replays a captured HIP
    graph instead of eager launches; tune: the library's autotuner picks each launch
    (kernel variant, tile length, grid) first, outside the timed region."""
    import numpy as np
    import torch

    ops = [M.MortarOperator([s]) for s in specs] if plain else [M.MortarOperator(specs)]
    t0 = time.time()
    base = []
    for i, spec in enumerate(specs):
        inp = W.make_inputs(spec, seed=2 + i, delta=disp(0)[i], noise=1e-4)
        base.append({k: None if v is None else torch.from_numpy(W.round_to(v, spec.precision)).cuda()
                     for k, v in inp.items()})
        del inp
    set_bytes = sum(algorithmic_bytes(s) for s in specs)
    nsets = max(2, int(np.ceil(rotate_bytes / set_bytes)))
    sets = []
    for r in range(nsets):
        per = []
        for spec, b in zip(specs, base):
            dt = torch.float64 if spec.precision == W.FP64 else torch.float32
            d = {k: None if v is None else v.clone() for k, v in b.items()}
            d["Fs"] = torch.zeros((5, spec.P, spec.n_face_static), dtype=dt, device="cuda")
            d["Fm"] = torch.zeros((5, spec.P, spec.n_face_moving), dtype=dt, device="cuda")
            per.append(d)
        sets.append(per)
    del base
    torch.cuda.synchronize()
    print(f"[bench] {'+'.join(s.name for s in specs)} prec={specs[0].precision} sets={nsets} x "
          f"{set_bytes / 1e6:.1f} MB graph={graph} plain={plain} (setup {time.time() - t0:.1f} s)",
          file=sys.stderr, flush=True)

    def args(per, sel=None):
        sel = range(len(specs)) if sel is None else sel
        return ([per[i]["Us"] for i in sel], [per[i]["Um"] for i in sel], [per[i]["Gs"] for i in sel],
                [per[i]["Gm"] for i in sel], [per[i]["Fs"] for i in sel], [per[i]["Fm"] for i in sel])

    tuning = None
    if fixed is not None:
        tuning = []
        for i, op in enumerate(ops):
            op.update([disp(0)[i]] if plain else disp(0))
            v, tiles, g = fixed
            tiles = tiles if len(tiles) == len(op.specs) else [tiles[0]] * len(op.specs)
            op.set_tuning([{"variant": v, "tile_len": t, "grid": g} for t in tiles])
            tuning += op.tuning()
        print(f"[bench] fixed tuning: {tuning}", file=sys.stderr, flush=True)
    elif tune:
        t1 = time.time()
        tuning = []
        for i, op in enumerate(ops):
            sel = [i] if plain else None
            op.update([disp(0)[i]] if plain else disp(0))
            tuning += op.autotune(*args(sets[0], sel), reps=3, cache=tune_cache)
        torch.cuda.synchronize()
        print(f"[bench] autotune {time.time() - t1:.2f} s: {tuning}", file=sys.stderr, flush=True)

    # per-stage conservation residual sums (FP64, on the device, no synchronization)
    cons_dev = [torch.zeros((1 if plain else len(specs), 5, 3), dtype=torch.float64, device="cuda")
                for _ in ops]

    # graph mode: one captured stage per buffer set, flux and conservation sums together
    graphs = None
    if graph:
        ops[0].update(disp(0))
        graphs = [ops[0].graph(*args(per), cons_out=cons_dev[0]) for per in sets]

    # eager stages with their arguments marshalled once per buffer set (update + flux +
    # conservation sums: three C calls per operator)
    stages = None if graph else [[op.stage(*args(per, [i] if plain else None), cons_out=cons_dev[i])
                                  for i, op in enumerate(ops)] for per in sets]

    def step(k):
        d = disp(k)
        if graph:
            graphs[k % nsets].launch(d)
        else:
            for i, st in enumerate(stages[k % nsets]):
                st([d[i]] if plain else d)

    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        step(warmup + k)
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / steps
    cs = torch.cat(cons_dev).cpu().numpy()
    step_cons_rel = float(np.max(np.abs(cs[:, :, 0] - cs[:, :, 1]) / cs[:, :, 2]))

    # the fused flux launch(es) alone, timed with HIP events on the stream they run on:
    # the average over a region of back-to-back launches (per-launch event pairs add the
    # events' own cost to every launch; they only give the spread)
    d = disp(warmup + steps)
    for i, op in enumerate(ops):
        op.update([d[i]] if plain else d)

    def flux_only(per):
        if plain:
            for i, op in enumerate(ops):
                op.flux(*args(per, [i]))
        else:
            ops[0].flux(*args(per))

    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    r0.record()
    for k in range(steps):
        flux_only(sets[k % nsets])
    r1.record()
    torch.cuda.synchronize()
    kavg = r0.elapsed_time(r1) / steps
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for k in range(steps):
        evs[k][0].record()
        flux_only(sets[k % nsets])
        evs[k][1].record()
    torch.cuda.synchronize()
    kms = np.array([a.elapsed_time(b) for a, b in evs])

    # the BR1 lifting surface term through the same operator (one launch per interface),
    # timed the same way; inputs rotate with the flux sets
    lift = None
    if measure_lifting:
        dt = torch.float64 if specs[0].precision == W.FP64 else torch.float32
        louts = [(torch.zeros((3, 5, sp.P, sp.n_face_static), dtype=dt, device="cuda"),
                  torch.zeros((3, 5, sp.P, sp.n_face_moving), dtype=dt, device="cuda")) for sp in specs]

        def lift_only(per):
            for i, op in enumerate(ops):
                sel = [i] if plain else range(len(specs))
                op.lifting([per[j]["Us"] for j in sel], [per[j]["Um"] for j in sel],
                           [louts[j][0] for j in sel], [louts[j][1] for j in sel])

        for k in range(3):
            lift_only(sets[k % nsets])
        torch.cuda.synchronize()
        r0.record()
        for k in range(steps):
            lift_only(sets[k % nsets])
        r1.record()
        torch.cuda.synchronize()
        lms = r0.elapsed_time(r1) / steps
        lbytes = sum(lifting_bytes(sp) for sp in specs)
        lift = {"kernel_ms_avg": lms, "bytes_per_launch": lbytes,
                "achieved_GBs": lbytes / (lms * 1e-3) / 1e9,
                "frac": lbytes / (lms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del louts
    cons = []
    for i, op in enumerate(ops):
        sel = [i] if plain else range(len(specs))
        c = op.conservation([sets[0][j]["Fs"] for j in sel], [sets[0][j]["Fm"] for j in sel])
        cons.append(c)
    cons = np.concatenate(cons, axis=0)
    cons_rel = float(np.max(np.abs(cons[:, :, 0] - cons[:, :, 1]) / cons[:, :, 2]))
    if graphs:
        for g in graphs:
            g.close()
    for op in ops:
        op.close()
    pts = sum(s.mortar_points for s in specs)
    achieved = set_bytes / (kavg * 1e-3) / 1e9
    return {
        "pts_per_s": pts / (ms_step * 1e-3),
        "ms_per_step": ms_step,
        "kernel_ms_avg": kavg,
        "kernel_ms_median_event_pair": float(np.median(kms)),
        "kernel_ms_min_event_pair": float(np.min(kms)),
        "kernel_ms_max_event_pair": float(np.max(kms)),
        "kernel_pts_per_s": pts / (kavg * 1e-3),
        "bytes_per_launch": set_bytes,
        "achieved_GBs": achieved,
        "frac": achieved / HBM_PEAK_GBS,
        "conservation_rel_residual": cons_rel,
        "lifting": lift,
        "conservation_rel_residual_last_step": step_cons_rel,
        "rotated_sets": nsets,
        "tuning": tuning,
    }


def rel_err_per_var(spec, F_gpu, F_ref):
    """Per output variable: max |F_gpu - F_ref| over both sides' interface columns, over
    max(max |F_ref_v|, 1e-3 max_v' max |F_ref_v'|)."""
    import numpy as np
    cs, cm = spec.face_id_static.ravel(), spec.face_id_moving.ravel()
    g = [F_gpu[0][:, :, cs], F_gpu[1][:, :, cm]]
    r = [F_ref[0][:, :, cs], F_ref[1][:, :, cm]]
    scale = np.array([max(np.abs(r[0][v]).max(), np.abs(r[1][v]).max()) for v in range(5)])
    floor = 1e-3 * scale.max()
    return [float(max(np.abs(g[0][v] - r[0][v]).max(), np.abs(g[1][v] - r[1][v]).max())
                  / max(scale[v], floor)) for v in range(5)]


def host_cpu():
    """Host CPU facts for the baseline: the model name, the processor count the OS
    reports, the processors this process may run on, and the thread count a pool should
    use (the affinity count, capped by OMP_NUM_THREADS when that is set)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = os.cpu_count() or 1
    threads = affinity
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        threads = min(threads, int(omp))
    return {"model": model, "nproc": affinity, "os_cpu_count": os.cpu_count(),
            "threads": max(1, threads)}


def cpu_baseline(M, W, specs, disp, stages, target_s=12.0):
    """The FP64 oracle as it stands on whole stages of the workload (every interface of
    it; inputs as the GPU sees them, promoted to FP64), timed twice on this host: one
    thread, then the same routine over row ranges on every usable core (rows are
    independent periodic chains).  Each leg runs about target_s seconds of work unless
    stages is given.  The last stage is also run on the GPU in the headline precision to
    report the error per output variable of each interface."""
    from oracle import oracle as O
    import numpy as np
    import torch

    cpu = host_cpu()
    f64 = []
    for i, spec in enumerate(specs):
        inp = W.make_inputs(spec, seed=2 + i, delta=disp(1)[i], noise=1e-4)
        f64.append({k: None if v is None else np.asarray(W.round_to(v, spec.precision), dtype=np.float64)
                    for k, v in inp.items()})
        del inp
    pts = sum(s.mortar_points for s in specs)

    def leg(threads):
        t0 = time.perf_counter()
        k, refs = 0, None
        while True:
            k += 1
            refs = []
            for i, spec in enumerate(specs):
                n, s = O.decompose(disp(k)[i], spec.l_par)
                refs.append(O.mortar_flux(spec, n, s, f64[i]["Us"], f64[i]["Um"], f64[i]["Gs"],
                                          f64[i]["Gm"], threads=threads))
            el = time.perf_counter() - t0
            print(f"[bench] oracle stage {k}, {threads} thread(s) ({el:.1f} s)", file=sys.stderr,
                  flush=True)
            if (stages > 0 and k >= stages) or (stages <= 0 and el * (k + 1) / k > target_s):
                return k, el, refs

    k1, el1, _ = leg(1)
    kn, eln, refs = leg(cpu["threads"])
    errs = []
    op = M.MortarOperator(specs)
    try:
        dev, outs = [], []
        for i, spec in enumerate(specs):
            dev.append({key: None if v is None else
                        torch.from_numpy(np.ascontiguousarray(W.round_to(v, spec.precision))).cuda()
                        for key, v in f64[i].items()})
            dt = torch.float64 if spec.precision == W.FP64 else torch.float32
            outs.append((torch.zeros((5, spec.P, spec.n_face_static), dtype=dt, device="cuda"),
                         torch.zeros((5, spec.P, spec.n_face_moving), dtype=dt, device="cuda")))
        op.update(disp(kn))
        op.flux([d["Us"] for d in dev], [d["Um"] for d in dev], [d["Gs"] for d in dev],
                [d["Gm"] for d in dev], [o[0] for o in outs], [o[1] for o in outs])
        torch.cuda.synchronize()
        for spec, o, ref in zip(specs, outs, refs):
            errs.append(rel_err_per_var(spec, (o[0].double().cpu().numpy(), o[1].double().cpu().numpy()), ref))
    finally:
        op.close()
    names = " + ".join(s.name for s in specs)
    return {"value": kn * pts / eln, "unit": "mortar points/s", "cores": cpu["threads"],
            "kind": "oracle",
            "sample": f"{kn} whole stages of {names} ({pts} mortar points per stage; FP64 oracle, "
                      f"rows split over {cpu['threads']} threads, {eln:.1f} s)",
            "single_thread": {"value": k1 * pts / el1, "cores": 1,
                              "sample": f"{k1} whole stages, one thread, {el1:.1f} s"},
            "host": cpu,
            "gpu_rel_err_per_var": errs}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the operator is "
                                   "single-GPU (multi-GPU sharding is a design note only)",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    if a.copy_calibration > 0:
        torch.cuda.set_device(0)
        copy_calibration(a.copy_calibration)
        return
    if a.stream_reference > 0:
        torch.cuda.set_device(0)
        stream_reference(a.stream_reference)
        return

    from paper_2008_04356_amd import mortar as M
    from paper_2008_04356_amd import workloads as W

    torch.cuda.set_device(0)
    prec = {"fp32": W.FP32, "bf16": W.BF16_MFMA, "fp16": W.FP16_MFMA}[a.precision]
    specs32, disp = W.config(a.config, precision=prec)
    graph = (a.graph or len(specs32) > 1) and not a.eager
    fixed = None
    if a.tuning is not None:
        v, t, g = a.tuning.split(",")
        fixed = (int(v), [int(x) for x in t.split("/")], int(g))
    r32 = run_leg(M, W, specs32, disp, a.steps, a.warmup, a.rotate_bytes, graph=graph,
                  tune=not a.no_autotune, tune_cache=a.tune_cache, fixed=fixed,
                  measure_lifting=not a.no_lifting)
    r64 = None
    if not a.no_fp64:
        specs64, _ = W.config(a.config, precision=W.FP64)
        # the comparison point: plain FP64, one launch per interface
        r64 = run_leg(M, W, specs64, disp, a.steps, a.warmup, a.rotate_bytes, plain=True,
                      tune=not a.no_autotune, tune_cache=a.tune_cache)
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(M, W, specs32, disp, a.cpu_stages)
    kargs = {1: "<float,4,Euler,LF>", 2: "<float,6,NS,Roe>", 3: "<float,8,NS+metrics,Roe>",
             4: "<float,NS,Roe,N=3,5,7>", 5: "<float,10,Euler,Roe>",
             6: "<float,8,NS+metrics,Roe>", 7: "<float,8,NS+metrics,Roe>"}
    tuned = r32["tuning"][0]["variant"] if r32["tuning"] else 0
    if len(specs32) > 1:
        kernel = ("k_mortar_flux_rd_batch" if tuned == 2 else "k_mortar_flux_batch") + kargs[a.config]
    else:
        kernel = KERNEL_OF_VARIANT.get(tuned, "?") + " " + kargs.get(a.config, "")
    spec = specs32[0]
    names = {2: f"plane sliding interface N={spec.N}, {spec.n_par}x{spec.n_perp} face pairs, "
                "Navier-Stokes Roe+BR1 (mu=1e-4), displacement 0.0137 l_par per stage, FP32",
             3: f"plane annular axial interface N={spec.N}, {spec.n_par}x{spec.n_perp} face pairs, "
                "per-point metrics, Navier-Stokes Roe+BR1, FP32",
             4: "turbine-like batch: annulus N=7 320x125 + annulus N=5 256x72 + plane N=3 64x32, "
                "Navier-Stokes Roe+BR1, FP32, one persistent launch per stage"
                + (" (HIP graph)" if graph else ""),
             1: f"plane interface N={spec.N}, {spec.n_par}x{spec.n_perp}, Euler LF, FP32",
             5: f"plane interface N={spec.N}, {spec.n_par}x{spec.n_perp}, Euler Roe, FP32",
             6: f"cylindrical radial interface N={spec.N}, {spec.n_par}x{spec.n_perp} face pairs, "
                "polynomial face geometry, per-point metrics, Navier-Stokes Roe+BR1, FP32",
             7: f"conical interface (30 deg) N={spec.N}, {spec.n_par}x{spec.n_perp} face pairs, "
                "polynomial face geometry, per-point metrics, Navier-Stokes Roe+BR1, FP32"}
    # a plain device copy timed in the same process after the measured region: the
    # fraction of what a copy reaches, reported beside the fraction of the published peak
    copy_gbs = stream_rates(1.0, legs=("copy",))["copy_GBs"]
    traffic = measured_traffic(a.config, a.precision, r32["tuning"])
    out = {
        "metric": "mortar flux points/sec and HBM GB/s vs peak, batched FP32 vs plain FP64",
        "value": r32["pts_per_s"],
        "unit": "mortar points/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "f32 data, bf16 GEMM operands",
                  "fp16": "f32 data, f16 GEMM operands"}[a.precision],
        "data": "synthetic",
        "config": {"workload": names.get(a.config, f"config {a.config}"),
                   "mortar_points_per_step": sum(s.mortar_points for s in specs32),
                   "fp64": None if r64 is None else {
                       "value": r64["pts_per_s"], "ms_per_step": r64["ms_per_step"],
                       "kernel_ms_avg": r64["kernel_ms_avg"], "achieved_GBs": r64["achieved_GBs"],
                       "frac": r64["frac"],
                       "conservation_rel_residual": r64["conservation_rel_residual"],
                       "tuning": r64["tuning"]},
                   "fp32_kernel": {k: r32[k] for k in ("kernel_ms_avg", "kernel_ms_median_event_pair",
                                                       "kernel_ms_min_event_pair",
                                                       "kernel_ms_max_event_pair",
                                                       "kernel_pts_per_s",
                                                       "conservation_rel_residual",
                                                       "rotated_sets", "tuning")},
                   "lifting": r32["lifting"]},
        "roofline": {"bound": "hbm", "achieved": r32["achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": r32["frac"],
                     "traffic": traffic,
                     # the counters' bytes over the same average launch duration
                     "traffic_GBs": None if traffic is None
                     else traffic / (r32["kernel_ms_avg"] * 1e-3) / 1e9,
                     "kernel": kernel,
                     "bytes_per_launch": r32["bytes_per_launch"],
                     "measured_copy_GBs": copy_gbs,
                     "frac_of_measured_copy": r32["achieved_GBs"] / copy_gbs},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
