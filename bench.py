"""Benchmark of the fused active-LBM step on one MI355X.

Headline workload: the CIL model on five periodic 1024 x 1024 D2Q7 lattices
in FP32, one per mean density 0.5, 0.75, 1.0, 1.25, 1.5 (the paper's CIL
parameters A = 2, B = 0.3, tau = 1, sigma = 1/70 rescaled by lambda = 4 to
A = 0.125, sigma = 4/70), Gaussian polarisation noise (std 0.05) about +x.
One timed step advances all five lattices by one lattice Boltzmann step; the
five lattices run as one batch (lbm_sweep_batch with its tuned work tile:
two steps per launch on 64 x 16 tiles, graphs of up to 1024 steps), with the
FP64 observables sampled once at the end of the timed steps.  Inputs are
synthetic, seeded and resident in HBM before timing starts.

Prints one JSON line: MLUPS (million lattice-site updates per second), the
roofline of the dominant kernel (the two-step kernel against the VALU issue
peak, with its HBM bytes beside it; a one-step kernel against the 8 TB/s HBM3E
peak at 56 B per site-update in FP32, 28 B in the 16-bit deviation
storages), variants (one step per launch, per-lattice launches, 4096^2 in
FP32 / BF16 / FP16, MIPS, the square-lattice (D2Q9) variant at 72 B per
site-update, a 256-lattice batched phase sweep against the same lattices run
one by one, the learned surrogate, the paper's measurement protocol) and the
FP64 oracle timed on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BYTES_PER_SITE = {0: 56, 1: 28, 2: 28, 3: 32}
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions/s
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU lane-instructions per site-update of the fused CIL step (FP32, tau 1,
# noise on): SQ_INSTS_VALU / SQ_WAVES of the one-step kernel with one site
# per lane.  valu_per_site_update() reads the current figure from the counter
# summary in profiles/; this is the last measured value, used when that
# summary was taken on other kernel sources.
VALU_PER_SITE_UPDATE = 185
# the same for the square lattice (D2Q9): the one-step batch kernel with one
# site per lane (256 x 1 tiles), CIL, FP32, tau 1, noise on
Q9_VALU_PER_SITE_UPDATE = 223
# MIPS, two steps per launch on 64 x 16 tiles (4096^2, FP32, tau 2, noise
# on): every VALU instruction of the launch (both rings included) per
# site-update of the tile
MIPS2_VALU_PER_SITE_UPDATE = 267
# the same on the square lattice (D2Q9)
MIPS2_Q9_VALU_PER_SITE_UPDATE = 308


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="cil1024x5",
                    choices=["cil1024x5", "cil4096", "mips4096", "q9_cil4096", "q9_mips4096"],
                    help="mips4096: the 64 x 64 MIPS workload's parameters on 4096 x 4096; q9_*: the "
                         "square-lattice (D2Q9) variant; lbm_step unless --mode batch (the batched path, "
                         "two steps per launch where tuned)")
    ap.add_argument("--storage", type=int, default=0,
                    help="0 f32, 1 bf16 deviations, 2 fp16 deviations, 3 bf16 deviations with a float32 rest plane")
    ap.add_argument("--mode", default=None, choices=["batch", "single"],
                    help="default: batch for the D2Q7 CIL workloads in FP32, single (lbm_step) otherwise")
    ap.add_argument("--quick", action="store_true", help="headline measurement only (no variants)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=24,
                    help="oracle steps of the 1024^2 single-thread baseline run x 6 (default: 4 steps)")
    ap.add_argument("--tile-rows", type=int, default=0,
                    help="batch work tile: 0 tuned, 1/2/4 one step per launch, 8/16 two steps per launch, 1024 lattices resident in LDS")
    ap.add_argument("--launch", default="direct", choices=["direct", "graph"],
                    help="batch mode: launch every kernel of the timed sweep directly (default) or replay "
                         "captured graphs")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 7 x 1024 x 1024 float buffer --steps times (counter calibration)")
    return ap.parse_args()


def cpu_mips64(steps=1000):
    """FP64 oracle on the MIPS 64 x 64 configuration (1000 steps)."""
    import oracle as O
    import synth_inputs as SI
    cfg = SI.mips_small()
    ini = cfg.pop("init")
    p = O.make_params(cfg["nx"], cfg["ny"], cfg["model"], cfg["tau"], cfg["sigma"], cfg["A"], cfg["B"], cfg["C"],
                      cfg["rho_star"], cfg["u_max"], cfg["seed"])
    f = O.initialise(p, **ini)
    t0 = time.perf_counter()
    O.run(p, f, steps)
    dt = time.perf_counter() - t0
    return {"MLUPS": round(cfg["nx"] * cfg["ny"] * steps / dt / 1e6, 3), "seconds": round(dt, 3), "cores": 1,
            "sample": f"MIPS 64x64, {steps} steps, FP64, single thread"}


def host_cpu():
    """(model name, logical CPUs of the machine, threads this process may use:
    its CPU affinity, capped by OMP_NUM_THREADS when that is set)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        threads = min(threads, int(env))
    return model, os.cpu_count(), max(1, threads)


def cpu_baseline(steps):
    """FP64 oracle on the CIL workload's parameters at 64^2, 256^2 and 1024^2
    sites, on one host thread (the plain build) and on every thread this
    process may use (the OpenMP build: rows of a step in parallel, the same
    per-site arithmetic).  Each run takes about 4 M site-updates single
    threaded (4x that on all threads), a few seconds in all.  value: all
    threads at 1024^2, the benchmark's lattice size."""
    import oracle as O
    import synth_inputs as SI
    model, ncpu, threads = host_cpu()
    table = {}
    for n, s1 in ((64, 1000), (256, 64), (1024, max(1, steps // 6))):
        cfg = dict(SI.cil_1024(1.0), nx=n, ny=n)
        ini = cfg.pop("init")
        p = O.make_params(cfg["nx"], cfg["ny"], cfg["model"], cfg["tau"], cfg["sigma"], cfg["A"], cfg["B"],
                          cfg["C"], cfg["rho_star"], cfg["u_max"], cfg["seed"])
        f0 = O.initialise(p, **ini)
        row = {}
        for th, st in ((1, s1), (threads, s1 * 4)):
            f = f0.copy()
            t0 = time.perf_counter()
            if th == 1:
                O.run(p, f, st)
                used = 1
            else:
                used = O.run_parallel(p, f, st, th)
            dt = time.perf_counter() - t0
            row[str(used)] = {"MLUPS": round(n * n * st / dt / 1e6, 3), "steps": st, "seconds": round(dt, 3)}
        table[f"{n}x{n}"] = row
    top = table["1024x1024"][str(threads)] if str(threads) in table["1024x1024"] else \
        list(table["1024x1024"].values())[-1]
    return {"value": top["MLUPS"], "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": (f"one 1024x1024 CIL lattice (mean density 1.0) for {top['steps']} steps, FP64, "
                       f"{threads} host threads (OpenMP over rows); the table gives 1 and {threads} threads "
                       "at 64^2, 256^2 and 1024^2"),
            "host_cpu_model": model, "host_logical_cpus": ncpu, "threads_available": threads,
            "by_size_and_threads": table}


def cpu_q9(steps):
    """FP64 square-lattice (D2Q9) oracle, single thread, on a 1024 x 1024
    lattice with the CIL parameters of the D2Q9 workload."""
    import oracle as O
    from oracle import q9
    import synth_inputs as SI
    cfg = SI.q9_cil_4096(n=1024)
    ini = cfg.pop("init")
    p = O.make_params(cfg["nx"], cfg["ny"], cfg["model"], cfg["tau"], cfg["sigma"], cfg["A"], cfg["B"], cfg["C"],
                      cfg["rho_star"], cfg["u_max"], cfg["seed"])
    f = q9.initialise(p, **ini)
    t0 = time.perf_counter()
    q9.run(p, f, steps)
    dt = time.perf_counter() - t0
    return {"value": round(cfg["nx"] * cfg["ny"] * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": 1,
            "kind": "oracle",
            "sample": f"one 1024x1024 D2Q9 CIL lattice (mean density 0.74) for {steps} steps, FP64, single thread"}


def gparams(L, c, storage=0, rho_ref=0.0, lattice=0):
    return L.make_params(c["nx"], c["ny"], c["model"], c["tau"], c["sigma"], c["A"], c["B"], c["C"], c["rho_star"],
                         c["u_max"], c["seed"], storage=storage, rho_ref=rho_ref, lattice=lattice)


def make_lattices(L, cfgs, storage=0, lattice=0):
    lats = []
    for c in cfgs:
        c = dict(c)
        ini = c.pop("init")
        lats.append(L.Lattice(gparams(L, c, storage, ini["rho_mean"], lattice), init=L.make_init(**ini)))
    return lats


def time_single(L, torch, cfgs, steps, warmup, storage=0, lattice=0):
    """Each lattice stepped by lbm_step (one launch per lattice per step)."""
    lats = make_lattices(L, cfgs, storage, lattice)
    for lat in lats:
        lat.step(warmup)
        # lbm_step replays a graph of 64 steps captured on first use: capture
        # it (an even count keeps the buffer parity) before timing
        lat.step(64)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for lat in lats:
        lat.step(steps)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    obs = [lat.observables() for lat in lats]
    for lat in lats:
        lat.close()
    return ms, obs


def time_batch(L, torch, cfgs, steps, warmup, tile_rows=0, lattice=0, storage=0, use_graph=1):
    """All lattices advanced by lbm_sweep_batch (one launch per step, or per
    two steps for the two-step tiles), replaying captured graphs (use_graph
    1) or launching every kernel directly (0)."""
    lats = make_lattices(L, cfgs, storage, lattice)
    b = L.Batch([lat.params for lat in lats])
    for l, lat in enumerate(lats):
        b.set_state(l, lat.state)
        lat.close()
    # build the launch plan (tile-shape tuning and the captured graphs for
    # `steps` steps; no step runs), warm up, then prepare again: that only
    # moves each state into the first buffer of its pair, where a sweep
    # starts (after an odd warm-up it sits in the second), so the GPU idles
    # only briefly before the timed sweep
    b.run(steps, tile_rows=tile_rows, use_graph=2)
    b.run(warmup, tile_rows=tile_rows, use_graph=use_graph)
    b.run(steps, tile_rows=tile_rows, use_graph=2)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # the sweep is enqueued (its FP64 sample is computed on the GPU inside the
    # timed region) and its samples are read back after the timed region
    e0.record(s)
    b.run(steps, tile_rows=tile_rows, fetch=False, use_graph=use_graph)
    e1.record(s)
    torch.cuda.synchronize()
    out = b.samples()
    time_batch.tile_rows = tile_rows or L.lbm_sweep_tile_rows(b.params, b.n)
    # each chunk runs lattice group by lattice group (groups sized for the
    # Infinity Cache): a pass over the batch is that many kernel launches
    time_batch.groups = 1 if time_batch.tile_rows == L.LBM_TILE_RESIDENT else L.lbm_sweep_groups(b.params, b.n)
    return e0.elapsed_time(e1), [o[-1] for o in out]


CHUNK = 1024  # steps per captured graph in lbm_sweep_batch


def batch_launches(steps, rows):
    """(two-step launches, one-step launches) of an unsampled sweep of `steps`
    steps with work-tile rows `rows`: the same schedule lbm_sweep_batch
    builds (graphs of at most CHUNK steps; in each, an even number of
    two-step launches, then one-step launches for the rest)."""
    if rows < 8:
        return 0, steps
    two = one = 0
    left = steps
    while left > 0:
        c = min(left, CHUNK)
        q = c // 2
        q -= q & 1
        two += q
        one += c - 2 * q
        left -= c
    return two, one


def copy_probe(torch, copies):
    """A plain copy of 7 x 1024 x 1024 floats (28 MiB read, 28 MiB written)
    `copies` times: the known-size kernel the HBM counters are scaled by."""
    a = torch.rand((7, 1024, 1024), device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(copies):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"copy_probe": {"bytes_read_per_copy": a.numel() * 4, "bytes_written_per_copy": b.numel() * 4,
                           "copies": copies}}


# the sources the batched step kernels are built from (their bodies, the
# parameters the host prepares for them, and the launch code)
KERNEL_SOURCES = ("batch.hip", "capi.hip", "device.h", "internal.h")
# sources of the square-lattice (D2Q9) step kernels
Q9_SOURCES = ("q9.hip", "device_q9.h", "device.h", "capi.hip", "internal.h")
# sources of the batched D2Q9 kernels
KERNEL_SOURCES_Q9B = ("batch.hip", "device_q9.h", "device.h", "capi.hip", "internal.h")
# sources of the single-lattice D2Q7 step kernels (lbm_step)
STEP_SOURCES = ("step.hip", "device.h", "capi.hip", "internal.h")


def source_fingerprint(files=KERNEL_SOURCES):
    """sha256 over a kernel's sources (names and contents)."""
    h = hashlib.sha256()
    for name in files:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_1902_00530_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(name, files=KERNEL_SOURCES):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the kernel sources as they are now (else None)."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("source_sha256") != source_fingerprint(files):
        return None
    return c


def attach_traffic(r, name, files, sites, per_launch_s):
    """Fill roofline r's traffic from a committed counter summary of the same
    kernel sources and lattice size."""
    c = measured_traffic(name, files)
    if c is not None and c.get("sites") == sites:
        r["traffic"] = round(c["traffic_bytes_per_launch"] / per_launch_s / 1e9, 1)
        r["traffic_bytes_per_launch"] = c["traffic_bytes_per_launch"]
        r["traffic_vs_algorithmic"] = round(c["traffic_bytes_per_launch"] / c["algorithmic_bytes_per_launch"], 4)
    return r


def valu_per_site_update():
    """The per-unit VALU figure of the ALU roofline: SQ_INSTS_VALU x 64 /
    site-updates of the one-step kernel (one site per lane) from its committed
    counter summary when that was taken on the current kernel sources, else
    the last measured value (VALU_PER_SITE_UPDATE).  Returns (value, source)."""
    c = measured_traffic("counters_k_batch_step_1_cil_5x1024.json")
    if c is not None and c.get("valu_lane_instructions_per_site_update"):
        return float(c["valu_lane_instructions_per_site_update"]), "counters_k_batch_step_1_cil_5x1024.json"
    return float(VALU_PER_SITE_UPDATE), "stated (counter summary taken on other kernel sources)"


def roofline_two_step(sites, per_launch_s, kernel, rows, total_sites=None):
    """Two steps per launch: 2 x sites site-updates of VALU work against the
    VALU issue peak; the HBM side is the state read and written once.  sites:
    the sites one launch covers on average (a lattice group's share of the
    batch, total_sites)."""
    vpu, vsrc = valu_per_site_update()
    tops = vpu * 2 * sites / per_launch_s / 1e12
    hbm = BYTES_PER_SITE[0] * sites / per_launch_s / 1e9
    r = {"bound": "alu", "achieved": round(tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
         "unit": "T VALU lane-instructions/s", "frac": round(tops / VALU_PEAK_TOPS, 4), "traffic": None,
         "kernel": kernel, "avg_launch_us": round(per_launch_s * 1e6, 3),
         "valu_per_site_update": vpu, "valu_per_site_update_source": vsrc, "site_updates_per_launch": round(2 * sites),
         "hbm": {"achieved": round(hbm, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                 "frac": round(hbm / HBM_PEAK_GBPS, 4), "bytes_per_launch": BYTES_PER_SITE[0] * sites},
        "state_residency": ("Infinity Cache: lattice groups of at most 240 MiB keep their two buffers in the "
                            "256 MiB cache across a chunk's launches, so these bytes are not HBM traffic; the "
                            "step's HBM roofline is the line's hbm_roofline (4096^2, one step per launch)")}
    c = measured_traffic(f"counters_k_batch_step2_{rows}_cil_5x1024.json")
    if c is not None and c.get("sites") == (total_sites or sites):
        r["traffic"] = round(c["traffic_bytes_per_launch"] / per_launch_s / 1e9, 1)
        r["traffic_unit"] = "GB/s (measured bytes past the L2 per launch / avg launch)"
        r["traffic_bytes_per_launch"] = c["traffic_bytes_per_launch"]
        r["traffic_vs_algorithmic"] = round(c["traffic_bytes_per_launch"] / c["algorithmic_bytes_per_launch"], 4)
    return r


def roofline_mips_two_step(sites, per_launch_s, kernel, q=7):
    """MIPS, two steps per launch (64 x 16 tiles; q = 7 triangular, 9 square
    lattice): 2 x sites site-updates of VALU work at the kernel's own count
    per update (from its counter summary when taken on the current sources)
    against the VALU issue peak; the HBM side is the state read and written
    once per launch (56 or 72 B per site)."""
    name = "counters_k_batch_step2_mips_16_4096.json" if q == 7 else "counters_k_batch_step2_mips_q9_16_4096.json"
    c = measured_traffic(name, KERNEL_SOURCES if q == 7 else KERNEL_SOURCES_Q9B)
    if c is not None and c.get("sites") == sites and c.get("valu_lane_instructions_per_site_update"):
        vpu, vsrc = float(c["valu_lane_instructions_per_site_update"]), name
    else:
        vpu = float(MIPS2_VALU_PER_SITE_UPDATE if q == 7 else MIPS2_Q9_VALU_PER_SITE_UPDATE)
        vsrc = "stated (counter summary taken on other kernel sources)"
    tops = vpu * 2 * sites / per_launch_s / 1e12
    per_site = BYTES_PER_SITE[0] * q // 7
    hbm = per_site * sites / per_launch_s / 1e9
    r = {"bound": "alu", "achieved": round(tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
         "unit": "T VALU lane-instructions/s", "frac": round(tops / VALU_PEAK_TOPS, 4), "traffic": None,
         "kernel": kernel, "avg_launch_us": round(per_launch_s * 1e6, 3),
         "valu_per_site_update": vpu, "valu_per_site_update_source": vsrc, "site_updates_per_launch": round(2 * sites),
         "hbm": {"achieved": round(hbm, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                 "frac": round(hbm / HBM_PEAK_GBPS, 4), "bytes_per_launch": per_site * sites}}
    if c is not None and c.get("sites") == sites and c.get("traffic_bytes_per_launch"):
        r["traffic"] = round(c["traffic_bytes_per_launch"] / per_launch_s / 1e9, 1)
        r["traffic_bytes_per_launch"] = c["traffic_bytes_per_launch"]
        r["traffic_vs_algorithmic"] = round(c["traffic_bytes_per_launch"] / c["algorithmic_bytes_per_launch"], 4)
    return r


def q9_valu_per_site_update():
    """valu_per_site_update() of the D2Q9 one-step batch kernel (256 x 1
    tiles), from its counter summary when taken on the current sources."""
    c = measured_traffic("counters_k_batch_q9_step_1_cil_4096.json", KERNEL_SOURCES_Q9B)
    if c is not None and c.get("valu_lane_instructions_per_site_update"):
        return float(c["valu_lane_instructions_per_site_update"]), "counters_k_batch_q9_step_1_cil_4096.json"
    return float(Q9_VALU_PER_SITE_UPDATE), "stated (counter summary taken on other kernel sources)"


def roofline_q9_two_step(sites, per_launch_s, kernel):
    """D2Q9, two steps per launch: 2 x sites site-updates of VALU work (the
    one-step kernel's count per update) against the VALU issue peak; the HBM
    side is the state (72 B per site in FP32) read and written once."""
    vpu, vsrc = q9_valu_per_site_update()
    tops = vpu * 2 * sites / per_launch_s / 1e12
    hbm = 72 * sites / per_launch_s / 1e9
    return {"bound": "alu", "achieved": round(tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "T VALU lane-instructions/s", "frac": round(tops / VALU_PEAK_TOPS, 4), "traffic": None,
            "kernel": kernel, "avg_launch_us": round(per_launch_s * 1e6, 3),
            "valu_per_site_update": vpu, "valu_per_site_update_source": vsrc, "site_updates_per_launch": round(2 * sites),
            "hbm": {"achieved": round(hbm, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(hbm / HBM_PEAK_GBPS, 4), "bytes_per_launch": 72 * sites}}


def roofline(storage, sites_per_launch, per_launch_s, kernel, q=7):
    """HBM roofline of a one-step kernel: each site's q populations read once
    and written once (q = 7 triangular, 9 square lattice)."""
    per_site = BYTES_PER_SITE[storage] * q // 7
    achieved = per_site * sites_per_launch / per_launch_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None, "kernel": kernel,
            "bytes_per_site": per_site, "avg_launch_us": round(per_launch_s * 1e6, 3)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU only; multi-GPU runs are not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_1902_00530_amd as L
    import synth_inputs as SI

    torch.cuda.set_device(0)
    if args.copy_probe:
        print(json.dumps(copy_probe(torch, args.steps)), flush=True)
        return
    lattice, q = 0, 7
    if args.workload == "cil1024x5":
        cfgs = [SI.cil_1024(r, l) for l, r in enumerate(SI.CIL_DENSITIES)]
        wname = "CIL 5 x 1024x1024 periodic D2Q7, mean density 0.5..1.5 (x4 scaled), sigma 4/70, tau 1"
    elif args.workload == "cil4096":
        cfgs = [SI.cil_4096()]
        wname = "CIL 4096x4096 periodic D2Q7, mean density 0.74 (x4 scaled), sigma 4/70, tau 1"
    elif args.workload == "mips4096":
        cfgs = [dict(SI.mips_small(), nx=4096, ny=4096)]
        wname = "MIPS 4096x4096 periodic D2Q7, mean density 1.0 (x8 scaled), sigma 8/70, tau 2"
    elif args.workload == "q9_cil4096":
        cfgs, lattice, q = [SI.q9_cil_4096()], L.LBM_D2Q9, 9
        wname = "CIL 4096x4096 periodic D2Q9, mean density 0.74 (x4 scaled), sigma 4/70, tau 1"
    else:
        cfgs, lattice, q = [SI.q9_mips_4096()], L.LBM_D2Q9, 9
        wname = "MIPS 4096x4096 periodic D2Q9, mean density 1.0 (x8 scaled), sigma 8/70, tau 2"
    sites = sum(c["nx"] * c["ny"] for c in cfgs)
    mode = args.mode or ("batch" if args.workload in ("cil1024x5", "cil4096") else "single")

    t_wall = time.perf_counter()
    rows, ngr = 0, 1
    if mode == "batch":
        # Each step launch of these batches carries 25-45 us of GPU work, far
        # more than the host needs to issue it, and replaying a graph of the
        # same launches took 14-28 us more GPU time per 20-step call on this
        # ROCm: the timed sweep launches its kernels directly by default.
        ms, obs = time_batch(L, torch, cfgs, args.steps, args.warmup, args.tile_rows, lattice, args.storage,
                             use_graph=1 if args.launch == "graph" else 0)
        rows = time_batch.tile_rows
        ngr = time_batch.groups
        two, one = batch_launches(args.steps, rows)
        gtxt = f"; {ngr} lattice groups per pass" if ngr > 1 else ""
        if args.workload in ("mips4096", "q9_mips4096"):
            launches = (two + 0.5 * one if two else args.steps) * ngr
            lat_name = "D2Q9" if lattice else "D2Q7"
            kernel = (f"k_batch_step2_mips<{lat_name},F32,noisy,{rows}> (64x{rows} tiles, two steps per launch; "
                      f"{two} launches + {one} one-step launches + 1 FP64 sample)" if two else
                      f"{'k_batch_q9_step_mips' if lattice else 'k_batch_step_mips'}<F32,noisy> (one step per launch, "
                      f"+1 FP64 sample)")
        elif lattice:
            launches = (two + 0.5 * one if two else args.steps) * ngr
            kernel = (f"k_batch_q9_step2<CIL,unit-tau,noisy,{rows}> (64x{rows} tiles, two steps per launch{gtxt})"
                      if two else f"k_batch_q9_step (one step per launch, tile rows {rows}{gtxt})")
        elif two:
            # a one-step launch moves the same bytes as a two-step launch
            # and does half the site work: count it as half a launch
            launches = (two + 0.5 * one) * ngr
            kernel = (f"k_batch_step2<CIL,unit-tau,noisy,{rows}> (64x{rows} tiles, two steps per launch; "
                      f"{two * ngr} launches + {one * ngr} one-step launches + 1 FP64 sample{gtxt}; "
                      f"{'launched directly' if args.launch == 'direct' else 'captured graphs'})")
        else:
            launches = args.steps * ngr
            tile = {1: "256x1", 2: "128x2", 4: "64x4"}.get(rows, "?")
            kernel = f"k_batch_step<CIL,unit-tau,noisy>, tile {tile} (+1 FP64 sample at the end{gtxt})"
    else:
        ms, obs = time_single(L, torch, cfgs, args.steps, args.warmup, args.storage, lattice)
        st = {0: "F32", 1: "BF16dev", 2: "F16dev", 3: "BF16devR32"}[args.storage]
        launches = args.steps * len(cfgs)
        kernel = {"q9_cil4096": f"k_q9_step_local<CIL,{st},unit-tau,noisy,streamed stores>",
                  "q9_mips4096": f"k_q9_step_mips<{st},noisy,streamed stores>",
                  "mips4096": f"k_step_mips<{st},noisy,16,8,streamed stores>"}.get(
                      args.workload, f"k_step_local<CIL,{st},unit-tau,noisy,streamed stores>")
    wall = time.perf_counter() - t_wall
    per_launch = ms / 1e3 / launches
    mlups = sites * args.steps / (ms / 1e3) / 1e6
    line = {
        "metric": ("MLUPS of the fused MIPS step" if args.workload == "mips4096" else
                   "MLUPS of the fused CIL step (FP32) and % of HBM peak" if lattice == 0 else
                   f"MLUPS of the fused D2Q9 {'MIPS' if args.workload == 'q9_mips4096' else 'CIL'} step"),
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f32", 1: "bf16 storage, f32 math", 2: "f16 storage, f32 math",
                  3: "bf16 storage with f32 rest population, f32 math"}[args.storage],
        "data": "synthetic",
        "config": {"workload": wname, "lattices": len(cfgs), "sites": sites, "storage": args.storage,
                   "mode": mode, **({"tile_rows": rows, "lattice_groups": ngr, "launch": args.launch}
                                    if mode == "batch" else {})},
        "roofline": (roofline_mips_two_step(sites, per_launch, kernel, q)
                     if rows >= 8 and args.workload in ("mips4096", "q9_mips4096")
                     else roofline_two_step(sites / ngr, per_launch, kernel, rows, sites) if rows >= 8 and not lattice
                     else roofline(args.storage, sites / (launches / args.steps), per_launch, kernel, q)
                     if rows < 8 else roofline_q9_two_step(sites / ngr, per_launch, kernel)),
        "phi": [round(o["phi"], 6) for o in obs],
        "wall_s": round(wall, 3),
    }

    if args.workload == "q9_cil4096" and args.storage == 0:
        if mode == "single":
            attach_traffic(line["roofline"], "counters_k_q9_step_local_cil_4096.json", Q9_SOURCES, sites, per_launch)
        elif rows >= 8:
            attach_traffic(line["roofline"], f"counters_k_batch_q9_step2_{rows}_cil_4096.json", KERNEL_SOURCES_Q9B,
                           sites, per_launch)

    if args.workload == "mips4096" and args.storage == 0 and mode == "single":
        attach_traffic(line["roofline"], "counters_k_step_mips_4096.json", STEP_SOURCES, sites, per_launch)
    if args.workload == "cil4096" and args.storage == 0 and mode == "single":
        attach_traffic(line["roofline"], "counters_k_step_local_cil_4096.json", STEP_SOURCES, sites, per_launch)

    if mode == "batch" and args.workload == "cil1024x5" and args.storage == 0 and rows < 8:
        c = measured_traffic(f"counters_k_batch_step_{rows}_cil_5x1024.json")
        if c is not None and c.get("sites") == sites:
            line["roofline"]["traffic"] = round(c["traffic_bytes_per_launch"] / per_launch / 1e9, 1)
            line["roofline"]["traffic_bytes_per_launch"] = c["traffic_bytes_per_launch"]
            line["roofline"]["traffic_vs_algorithmic"] = round(
                c["traffic_bytes_per_launch"] / c["algorithmic_bytes_per_launch"], 4)

    if not args.quick and args.workload == "cil1024x5" and args.storage == 0:
        var = {}
        # the headline's timed sweep in the other launch form, same steps
        other = "graph" if args.launch == "direct" else "direct"
        mso, _ = time_batch(L, torch, cfgs, args.steps, args.warmup, args.tile_rows, lattice, args.storage,
                            use_graph=1 if other == "graph" else 0)
        var[f"cil1024x5_{other}_launches" if other == "direct" else "cil1024x5_graph_replay"] = {
            "MLUPS": round(sites * args.steps / (mso / 1e3) / 1e6, 1), "ms": round(mso, 4),
            "vs_headline": round(ms / mso, 4)}
        k = max(200, args.steps // 4)
        # the same batch with one step per launch (256 x 1 tiles): the plain
        # fused step against the HBM roofline
        ms_one, _ = time_batch(L, torch, cfgs, k, 20, tile_rows=1)
        ng1 = time_batch.groups
        per_one = ms_one / 1e3 / (k * ng1)
        r1 = roofline(0, sites / ng1, per_one, f"k_batch_step<CIL,unit-tau,noisy>, 256x1 tiles, {ng1} lattice groups")
        c = measured_traffic("counters_k_batch_step_1_cil_5x1024.json")
        if c is not None and c.get("sites") == sites:
            r1["traffic"] = round(c["traffic_bytes_per_launch"] / per_one / 1e9, 1)
            r1["traffic_vs_algorithmic"] = round(c["traffic_bytes_per_launch"] / c["algorithmic_bytes_per_launch"], 4)
        var["cil1024x5_one_step_per_launch"] = {"MLUPS": round(sites * k / (ms_one / 1e3) / 1e6, 1),
                                                "roofline": r1,
                                                "two_step_speedup": round((ms_one / k) / (ms / args.steps), 3)}
        ms1, _ = time_single(L, torch, cfgs, k, 20)
        var["cil1024x5_per_lattice_launches"] = {"MLUPS": round(sites * k / (ms1 / 1e3) / 1e6, 1),
                                                  "batch_speedup": round((ms1 / k) / (ms / args.steps), 3)}
        big = [SI.cil_4096()]
        nbig = big[0]["nx"] * big[0]["ny"]
        f32 = None
        for st, name in ((0, "f32"), (1, "bf16_dev"), (2, "f16_dev"), (3, "bf16_dev_r32")):
            msb, _ = time_single(L, torch, big, 200, 10, st)
            per = msb / 1e3 / 200
            r = roofline(st, nbig, per, f"k_step_local<CIL,{name},streamed stores>")
            v = {"MLUPS": round(nbig / per / 1e6, 1), "GBps": r["achieved"], "frac_hbm": r["frac"],
                 "avg_launch_us": r["avg_launch_us"]}
            if st == 0:
                f32 = per
                # the HBM roofline of the step: this lattice's state (940 MB)
                # streams from HBM every launch, unlike the headline batch's
                # lattice groups, which stay in the Infinity Cache
                attach_traffic(r, "counters_k_step_local_cil_4096.json", STEP_SOURCES, nbig, per)
                line["hbm_roofline"] = {
                    "workload": "CIL 4096x4096 FP32, lbm_step, one step per launch", "bound": "hbm",
                    "kernel": r["kernel"], "achieved": r["achieved"], "peak": r["peak"], "unit": r["unit"],
                    "frac": r["frac"], "traffic": r["traffic"],
                    "traffic_vs_algorithmic": r.get("traffic_vs_algorithmic"),
                    "bytes_per_site": r["bytes_per_site"], "avg_launch_us": r["avg_launch_us"],
                    "profile": "profiles/k_step_local_cil_4096.md"}
            else:
                v["speedup_vs_f32"] = round(f32 / per, 3)
                v["stated_error_vs_fp64"] = {
                    "bf16_dev": "100-step rel Linf 2.9e-3, mass drift 1.7e-3 / 2e4 steps",
                    "f16_dev": "100-step rel Linf 3.4e-4, mass drift 4.9e-5 / 2e4 steps",
                    "bf16_dev_r32": "100-step rel Linf and mass drift: see tests/test_precision_gpu.py"}[name]
            var["cil4096_" + name] = v
        # MIPS (density-dependent motility, LDS density halo): the 64 x 64
        # configuration (1000 steps) and the same parameters at 4096^2
        mcfg = SI.mips_small()
        msm, _ = time_single(L, torch, [mcfg], 1000, 20)
        var["mips64_1000_steps"] = {"MLUPS": round(64 * 64 * 1000 / (msm / 1e3) / 1e6, 2),
                                    "ms": round(msm, 3), "us_per_step": round(msm, 3),
                                    "note": "4,096 sites: one launch per step, launch-bound"}
        mbig = dict(mcfg, nx=4096, ny=4096)
        msb, _ = time_single(L, torch, [mbig], 100, 10)
        rm = roofline(0, 4096 * 4096, msb / 1e3 / 100, "k_step_mips<F32,noisy,16,8,streamed stores>")
        attach_traffic(rm, "counters_k_step_mips_4096.json", STEP_SOURCES, 4096 * 4096, msb / 1e3 / 100)
        var["mips4096_f32"] = {"MLUPS": round(4096 * 4096 * 100 / (msb / 1e3) / 1e6, 1), "GBps": rm["achieved"],
                               "frac_hbm": rm["frac"], "avg_launch_us": rm["avg_launch_us"],
                               "traffic_GBps": rm["traffic"], "traffic_vs_algorithmic": rm.get("traffic_vs_algorithmic")}
        # the same lattice through the batched path: two steps per launch
        # (k_batch_step2_mips, tuned among 64x4 one-step and 64x8 / 64x16
        # two-step tiles)
        msb2, _ = time_batch(L, torch, [mbig], 100, 10)
        var["mips4096_f32_two_step"] = {"MLUPS": round(4096 * 4096 * 100 / (msb2 / 1e3) / 1e6, 1),
                                        "tile_rows": time_batch.tile_rows,
                                        "speedup_vs_f32_one_step": round(msb / msb2, 3)}
        # the square lattice (D2Q9, 72 B per site-update in FP32): CIL in the
        # three storages and MIPS at 4096^2, one launch per step
        q9c = [SI.q9_cil_4096()]
        q9f32 = None
        for st, name in ((0, "f32"), (1, "bf16_dev"), (2, "f16_dev")):
            msq, _ = time_single(L, torch, q9c, 200, 10, st, lattice=L.LBM_D2Q9)
            per = msq / 1e3 / 200
            r = roofline(st, nbig, per, f"k_q9_step_local<CIL,{name},streamed stores>", q=9)
            v = {"MLUPS": round(nbig / per / 1e6, 1), "GBps": r["achieved"], "frac_hbm": r["frac"],
                 "avg_launch_us": r["avg_launch_us"], "bytes_per_site": r["bytes_per_site"]}
            if st == 0:
                attach_traffic(r, "counters_k_q9_step_local_cil_4096.json", Q9_SOURCES, nbig, per)
                if r["traffic"] is not None:
                    v["traffic_GBps"] = r["traffic"]
                    v["traffic_vs_algorithmic"] = r["traffic_vs_algorithmic"]
            if st == 0:
                q9f32 = per
            else:
                v["speedup_vs_f32"] = round(q9f32 / per, 3)
            var["q9_cil4096_" + name] = v
        # D2Q9 at 4096^2 through the batched path (tuned: two steps per launch)
        msq2, _ = time_batch(L, torch, q9c, 200, 10, lattice=L.LBM_D2Q9)
        var["q9_cil4096_f32_two_step"] = {"MLUPS": round(nbig * 200 / (msq2 / 1e3) / 1e6, 1),
                                          "tile_rows": time_batch.tile_rows,
                                          "speedup_vs_f32_one_step": round(q9f32 / (msq2 / 1e3 / 200), 3)}
        msq, _ = time_single(L, torch, [SI.q9_mips_4096()], 100, 10, lattice=L.LBM_D2Q9)
        rq = roofline(0, nbig, msq / 1e3 / 100, "k_q9_step_mips<F32,noisy,streamed stores>", q=9)
        var["q9_mips4096_f32"] = {"MLUPS": round(nbig * 100 / (msq / 1e3) / 1e6, 1), "GBps": rq["achieved"],
                                  "frac_hbm": rq["frac"], "avg_launch_us": rq["avg_launch_us"]}
        msq2m, _ = time_batch(L, torch, [SI.q9_mips_4096()], 100, 10, lattice=L.LBM_D2Q9)
        var["q9_mips4096_f32_two_step"] = {"MLUPS": round(nbig * 100 / (msq2m / 1e3) / 1e6, 1),
                                           "tile_rows": time_batch.tile_rows,
                                           "speedup_vs_f32_one_step": round(msq / msq2m, 3)}
        # FP32 at 4096^2 through the batched path (two steps per launch)
        ms2, _ = time_batch(L, torch, big, 200, 10)
        rows2 = time_batch.tile_rows
        var["cil4096_f32_two_step"] = {"MLUPS": round(nbig * 200 / (ms2 / 1e3) / 1e6, 1), "tile_rows": rows2,
                                       "speedup_vs_f32_one_step": round(f32 / (ms2 / 1e3 / 200), 3)}
        # 256-lattice batched phase sweep vs the same lattices one by one
        bcfgs = SI.batch_sweep()
        nb_sites = sum(c["nx"] * c["ny"] for c in bcfgs)
        kb = 100
        msb, _ = time_batch(L, torch, bcfgs, kb, 10)
        ms1, _ = time_single(L, torch, bcfgs, kb, 10)
        var["batch256_phase_sweep"] = {
            "lattices": len(bcfgs), "sites": nb_sites,
            "MLUPS_batched": round(nb_sites * kb / (msb / 1e3) / 1e6, 1),
            "MLUPS_one_by_one": round(nb_sites * kb / (ms1 / 1e3) / 1e6, 1),
            "speedup": round(ms1 / msb, 3),
            "field_error": "0 (batch members equal single runs bit for bit)"}
        # the same sweep with 16-bit deviation storage, batched, against the
        # plain FP32 form (one lattice per launch) and the FP32 batch
        for st, name in ((1, "bf16_dev"), (2, "f16_dev"), (3, "bf16_dev_r32")):
            ms16, _ = time_batch(L, torch, bcfgs, kb, 10, storage=st)
            var["batch256_phase_sweep_" + name] = {
                "MLUPS_batched": round(nb_sites * kb / (ms16 / 1e3) / 1e6, 1), "tile_rows": time_batch.tile_rows,
                "speedup_vs_fp32_one_by_one": round(ms1 / ms16, 3),
                "speedup_vs_fp32_batched": round(msb / ms16, 3),
                "field_error": ("members equal lbm_step runs in the same storage bit for bit; storage error vs the "
                                "FP64 oracle as stated for cil4096_" + name)}
        # the same sweep on the square lattice (D2Q9, tuned tiles)
        msb, _ = time_batch(L, torch, bcfgs, kb, 10, lattice=L.LBM_D2Q9)
        ms1, _ = time_single(L, torch, bcfgs, kb, 10, lattice=L.LBM_D2Q9)
        var["q9_batch256_phase_sweep"] = {
            "lattices": len(bcfgs), "sites": nb_sites, "tile_rows": time_batch.tile_rows,
            "MLUPS_batched": round(nb_sites * kb / (msb / 1e3) / 1e6, 1),
            "MLUPS_one_by_one": round(nb_sites * kb / (ms1 / 1e3) / 1e6, 1),
            "speedup": round(ms1 / msb, 3),
            "field_error": "0 (batch members equal single runs bit for bit)"}
        # the paper's MIPS batch: 12 lattices of 90 x 30 (six densities, two
        # repeats), 20000 steps, in each batch form
        mcf = [dict(nx=90, ny=30, model=SI.MIPS, tau=2.0, sigma=1.0 / 70.0, A=0.0, B=0.0, C=50.0, rho_star=0.2,
                    u_max=0.3, seed=SI.seed_for(11, l),
                    init=dict(mode=1, rho_mean=r, rho_spread=0.0, angle_std=0.0, u_mag=0.1, pop_noise=1e-3))
               for l, r in enumerate((0.06, 0.08, 0.10, 0.125, 0.15, 0.18) * 2)]
        forms = {}
        for name, rows in (("64x16_two_step", 16), ("64x4", 4), ("resident", L.LBM_TILE_RESIDENT), ("tuned", 0)):
            msr, _ = time_batch(L, torch, mcf, 20000, 1000, rows)
            forms[name] = {"us_per_step": round(msr * 1e3 / 20000, 3),
                           "MLUPS": round(12 * 2700 * 20000 / (msr / 1e3) / 1e6, 1)}
        forms["tuned"]["tile_rows"] = time_batch.tile_rows
        var["mips_paper_batch_12x90x30"] = forms
        # learned surrogate (coarse 32x32 fields of 256^2 lattices, k = 50)
        from paper_1902_00530_amd import surrogate as S
        r = S.recipe(SI.surrogate_grid(256, 11000), SI.surrogate_grid(256, 21000), SI.surrogate_grid(256, 31000),
                     coarse=8, k=50, warmup=2000, rounds=320, epochs=30, batch=64, lr=1e-3, jumps=20,
                     check_every=4)
        r.pop("network")
        var["surrogate_256_k50"] = r
        # the method's run-to-run spread at coarser cells (same lattices, k = 50)
        fl = {}
        for c in (8, 16, 32):
            fl[f"{c}x{c}_sites_per_cell"] = round(S.noise_floor(SI.surrogate_grid(256, 21000), c, 50, 2000), 5)
        var["surrogate_noise_floor_by_cell"] = fl
        # where the floor drops below the fixed bound of 1e-2 (32 x 32 sites
        # per cell) and just above it (16 x 16): the same recipe and sweeps
        for c in (16, 32):
            r = S.recipe(SI.surrogate_grid(256, 11000), SI.surrogate_grid(256, 21000), SI.surrogate_grid(256, 31000),
                         coarse=c, k=50, warmup=2000, rounds=320, epochs=30, batch=64, lr=1e-3, jumps=20,
                         check_every=4)
            r.pop("network")
            var[f"surrogate_256_k50_cell{c}"] = r
        # the paper's measurement protocol (180 x 60 lattices, its CIL
        # parameters): the hysteresis ramps at A = 2 (50 increasing and 50
        # decreasing runs) and a (rho, A) phase diagram (9 A values x 10
        # repeats, rho 0.05 .. 0.40 every 1e4 steps), every run a lattice of
        # one batch
        from paper_1902_00530_amd import protocol as P
        code = {"HD": "D", "HO": "O", "B": "b", "RB": "R", "none": "-"}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = P.hysteresis(repeats=50)
        torch.cuda.synchronize()
        th = time.perf_counter() - t0
        snap = {}
        for r in (0.105, 0.1425, 0.185, 0.2875):
            k = min(range(len(h["up"]["rho"])), key=lambda i: abs(h["up"]["rho"][i] - r))
            snap[str(r)] = h["up"]["regime"][k]
        upd = 2 * 50 * 180 * 60 * h["up"]["steps"]
        var["protocol_hysteresis_A2"] = {
            "runs": 100, "steps_per_run": h["up"]["steps"], "seconds": round(th, 3),
            "MLUPS": round(upd / th / 1e6, 1),
            "regimes_up": "".join(code[x] for x in h["up"]["regime"]),
            "regimes_down": "".join(code[x] for x in h["down"]["regime"]),
            "rho_from_to_step": [0.09, 0.35, 0.0025],
            "regime_at_paper_snapshot_densities": snap}
        A_vals = [0.0, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pd = P.phase_diagram(A_vals)
        torch.cuda.synchronize()
        tpd = time.perf_counter() - t0
        var["protocol_phase_diagram"] = {
            "runs": pd["lattices"], "steps_per_run": pd["steps"], "seconds": round(tpd, 3),
            "MLUPS": round(pd["lattices"] * 180 * 60 * pd["steps"] / tpd / 1e6, 1),
            "rho_from_to_step": [0.05, 0.40, 0.01],
            "regimes_by_A": {str(a): "".join(code[x] for x in row) for a, row in zip(A_vals, pd["regime"])}}
        # the paper's MIPS noise ramp (90 x 30, its MIPS parameter table, sigma
        # 1/70 -> 3/70 by 1/700), six mean densities x two runs in one batch;
        # relaxation and sampling shortened (paper: 1e6 steps, 100 samples
        # every 1e4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mr = P.mips_noise_ramp()
        torch.cuda.synchronize()
        tmr = time.perf_counter() - t0
        var["protocol_mips_noise_ramp"] = {
            "runs": mr["lattices"], "steps_per_run": mr["steps"], "seconds": round(tmr, 3),
            "MLUPS": round(mr["lattices"] * 90 * 30 * mr["steps"] / tmr / 1e6, 1),
            "sigma_from_to_step": [round(1 / 70, 6), round(3 / 70, 6), round(1 / 700, 6)],
            "steps_per_sigma": {"relax": 50000, "samples": 50, "sample_every": 1000},
            "regimes_by_rho": {str(r): "".join("P" if x == "PS" else "h" for x in row)
                               for r, row in zip(mr["rho"], mr["regime"])},
            "sigma_homogeneous_by_rho": {str(r): (round(x, 5) if x is not None else None)
                                         for r, x in zip(mr["rho"], mr["sigma_homogeneous"])}}
        line["variants"] = var
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_q9(args.cpu_steps) if lattice else cpu_baseline(args.cpu_steps)
        if not args.quick and not lattice:
            line["cpu_baseline"]["mips64_1000_steps"] = cpu_mips64()
            line["cpu_baseline"]["q9_cil1024"] = cpu_q9(10)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
