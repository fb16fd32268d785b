"""Benchmark of the fused active-LBM step on one MI355X.

Workload (default): the CIL model on five periodic 1024 x 1024 lattices in
FP32, one per mean density 0.5, 0.75, 1.0, 1.25, 1.5 (the paper's CIL
parameters A = 2, B = 0.3, tau = 1, sigma = 1/70 rescaled by lambda = 4),
initialised with Gaussian polarisation noise (std 0.05) about +x.  One timed
step advances all five lattices by one lattice Boltzmann step.  Inputs are
synthetic and seeded, resident in HBM before timing starts.

Prints one JSON line: MLUPS (million lattice-site updates per second), the
roofline of the fused step kernel (algorithmic 56 B per site-update against
the 8 TB/s HBM peak) and the FP64 oracle timed on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BYTES_PER_SITE = {0: 56, 1: 28, 2: 28}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="cil1024x5", choices=["cil1024x5", "cil4096"])
    ap.add_argument("--storage", type=int, default=0, help="0 f32, 1 bf16 deviations, 2 fp16 deviations")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=25)
    return ap.parse_args()


def cpu_baseline(steps):
    """FP64 oracle, single thread, on one lattice of the workload."""
    import oracle as O
    import synth_inputs as SI
    cfg = SI.cil_1024(1.0)
    ini = cfg.pop("init")
    p = O.make_params(cfg["nx"], cfg["ny"], cfg["model"], cfg["tau"], cfg["sigma"], cfg["A"], cfg["B"], cfg["C"],
                      cfg["rho_star"], cfg["u_max"], cfg["seed"])
    f = O.initialise(p, **ini)
    t0 = time.perf_counter()
    O.run(p, f, steps)
    dt = time.perf_counter() - t0
    return {"value": cfg["nx"] * cfg["ny"] * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"one 1024x1024 CIL lattice (mean density 1.0) for {steps} steps, FP64, single thread"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_1902_00530_amd as L
    import synth_inputs as SI

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.workload == "cil1024x5":
        cfgs = [SI.cil_1024(r, l) for l, r in enumerate(SI.CIL_DENSITIES)]
        wname = "CIL 5 x 1024x1024 periodic D2Q7, mean density 0.5..1.5 (x4 scaled), FP32 storage"
    else:
        cfgs = [SI.cil_4096()]
        wname = "CIL 4096x4096 periodic D2Q7, mean density 0.74 (x4 scaled)"
    lats = []
    for c in cfgs:
        ini = c.pop("init")
        p = L.make_params(c["nx"], c["ny"], c["model"], c["tau"], c["sigma"], c["A"], c["B"], c["C"],
                          c["rho_star"], c["u_max"], c["seed"], storage=args.storage, rho_ref=ini["rho_mean"])
        lats.append(L.Lattice(p, init=L.make_init(**ini)))
    sites = sum(c["nx"] * c["ny"] for c in cfgs)
    torch.cuda.synchronize()

    for lat in lats:
        lat.step(args.warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for lat in lats:
        lat.step(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    obs = [lat.observables() for lat in lats]
    for lat in lats:
        lat.close()

    launches = len(lats) * args.steps
    per_launch_s = ms / 1e3 / launches
    sites_per_launch = sites / len(lats)
    achieved = BYTES_PER_SITE[args.storage] * sites_per_launch / per_launch_s / 1e9
    mlups = sites * args.steps / (ms / 1e3) / 1e6
    line = {
        "metric": "MLUPS (fused CIL step, FP32) and % HBM peak",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {0: "f32", 1: "bf16-dev storage, f32 math", 2: "f16-dev storage, f32 math"}[args.storage],
        "data": "synthetic",
        "config": {"workload": wname, "lattices": len(lats), "sites": sites, "storage": args.storage},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                     "kernel": "k_step_local<CIL>", "bytes_per_site": BYTES_PER_SITE[args.storage],
                     "avg_launch_us": round(per_launch_s * 1e6, 3)},
        "wall_s": round(wall, 4),
        "phi": [round(o["phi"], 6) for o in obs],
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
