#!/usr/bin/env python3
"""Benchmark: one full particle step (detection, canonical order, rows,
colouring, warm start, PGS, integration, body forces, zone aggregates) of the
50,000-sphere bulldozing bed on one MI355X.

Workload: 50k spheres r = 0.03 m U(0.9, 1.1), rho 2000, mu 0.7, c_p 2 kPa,
poured over a 4 x 2 m floor with walls and settled on the GPU before timing;
a 1.5 x 0.05 x 0.6 m box blade cuts 0.2 m below the settled surface at 1 m/s;
dt = 1/60 s, 150 PGS sweeps, previous-step warm start.  Inputs are resident
in HBM when the timed region starts.

Prints one JSON line.  value = contacts * PGS sweeps / s over the whole step.
roofline: the persistent PGS kernel, algorithmic bytes (176 B per pair
contact-sweep, 128 B per boundary contact-sweep) / its event-timed duration.
cpu_baseline: the FP64 oracle (single thread) on a 50k-sphere jammed bed of the
same radius, a bounded sample of about 10-30 s.
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2011_00459_amd import scenegen as SG  # noqa: E402
from paper_2011_00459_amd import terrain as T  # noqa: E402

HBM_PEAK_GBS = 8000.0
PAIR_BYTES, BOUND_BYTES = 176, 128
# HBM traffic of one k_pgs launch on this workload, from the FETCH_SIZE and
# WRITE_SIZE counter runs scaled by a copy kernel of known size (see
# profiles/k_pgs_bed50k_hbm_traffic.md); valid only for the kernel source it
# was measured on, else reported as null.
PGS_TRAFFIC = {"kernels_sha256_prefix": "94dafd6c4e5392d2", "bytes_per_launch": 3.167e9,
               "profile": "profiles/k_pgs_bed50k_hbm_traffic.md"}


# The same for k_advect on the 256 x 256 x 128 voxel grid
# (profiles/k_advect_voxels256_kernel_trace.md), keyed to terrain_voxels.hip.
ADVECT_TRAFFIC = {"kernels_sha256_prefix": "92ca9f936e1a6af0", "bytes_per_launch": 0.3757e9,
                  "profile": "profiles/k_advect_voxels256_kernel_trace.md"}


def source_traffic(entry, source):
    import hashlib
    with open(os.path.join(ROOT, "paper_2011_00459_amd", "csrc", source), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return entry["bytes_per_launch"] if sha == entry["kernels_sha256_prefix"] else None


def pgs_traffic():
    import hashlib
    src = os.path.join(ROOT, "paper_2011_00459_amd", "csrc", "terrain_kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return PGS_TRAFFIC["bytes_per_launch"] if sha == PGS_TRAFFIC["kernels_sha256_prefix"] else None


def device_sync():
    hip = ctypes.CDLL("libamdhip64.so.7")
    rc = hip.hipDeviceSynchronize()
    if rc != 0:
        raise RuntimeError(f"hipDeviceSynchronize failed ({rc})")


def build_bed(args):
    spec = SG.bed_scene(seed=2, n=args.n, r0=0.03, spread=0.1, lx=4.0, ly=2.0, mu=0.7, c=2000.0,
                        sweeps=args.sweeps, tool="none")
    solids = float(np.sum(4.0 / 3.0 * np.pi * spec["r"] ** 3))
    est_top = solids / (4.0 * 2.0 * 0.6)
    blade = SG.box_blade(-1.6, est_top - 0.2, width=1.5, thick=0.05, height=0.6, vx=0.0)
    spec["bodies"] = spec["bodies"] + [blade]
    spec["warm_start"] = "prev"
    sc = T.scene_from_specs(spec, cap_contacts=16 * args.n)
    # eager launches (measured faster than step-graph replays: the bed's PGS
    # 8.97 against 9.54-9.60 ms, the batch 1.52e10 against 1.48e10 contact
    # sweeps/s, one box each); --launch graphs replays the step graphs, whose
    # phase events are nodes of the graphs.  The HIP events time the PGS
    # launch inside the timed region either way.
    sc.set_step_graphs(args.launch == "graphs")
    return sc, spec, blade, est_top


def settle(sc, spec, blade, steps):
    # pour and settle with fewer sweeps, blade static in place
    sc.step(steps, stats=False)
    st = sc.step(1)[0]
    p = sc.get_particles(0)
    top = float(np.percentile(p["x"][:, 2] + p["r"], 99.0))
    return st, top


def timed_steps(sc, k):
    """K steps, one at a time so that every step's contact count is known."""
    device_sync()
    t0 = time.perf_counter()
    tot_cs = 0
    tot_bytes_pgs = 0
    pgs_ms = 0.0
    stats = []
    for _ in range(k):
        st = sc.step(1)[0]
        ph = sc.get_phase_times()
        pairs, allc = st["pair_contacts"], st["contacts"]
        tot_cs += allc * st["sweeps"]
        tot_bytes_pgs += (pairs * PAIR_BYTES + (allc - pairs) * BOUND_BYTES) * st["sweeps"]
        pgs_ms += ph["pgs"]
        stats.append((st, ph))
    device_sync()
    t1 = time.perf_counter()
    return t1 - t0, tot_cs, tot_bytes_pgs, pgs_ms, stats


def cpu_baseline(args):
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import pyoracle as O
    nx, ny = 60, 30
    nz = max(1, int(round(args.n / (nx * ny))))
    spec = SG.jammed_bed(seed=21, nx=nx, ny=ny, nz=nz, r0=0.03, sweeps=args.sweeps)
    o = O.OracleScene(spec)
    t0 = time.perf_counter()
    cs = 0
    steps = 0
    while True:
        out = o.step()
        cs += out["contacts"] * out["sweeps"]
        steps += 1
        if time.perf_counter() - t0 > args.cpu_seconds or steps >= 8:
            break
    dt = time.perf_counter() - t0
    return dict(value=cs / dt, unit="contacts*sweeps/s", cores=1, kind="oracle",
                sample=f"{steps} FP64 oracle steps (single thread) of a {len(spec['x'])}-sphere jammed bed, "
                       f"r 0.03 m, {args.sweeps} sweeps, {out['contacts']} contacts/step")


def build_batched(args):
    specs = SG.batch_specs(seed=3000, n_envs=args.envs, sweeps=args.sweeps)
    mat = specs[0]["material"]
    specs = [dict(s, material=mat, warm_start="prev") for s in specs]
    nmax = max(len(s["x"]) for s in specs)
    sc = T.scene_from_specs(specs, cap_particles=nmax, cap_contacts=8 * nmax)
    # tools held still while the beds settle
    still = []
    for e, s in enumerate(specs):
        b = [dict(x, id=i) for i, x in enumerate(s["bodies"])]
        moving = [dict(x) for x in b]
        for x in b:
            x["linvel"] = (0.0, 0.0, 0.0)
        sc.set_kinematic_bodies(e, b)
        still.append(moving)
    return sc, specs, still


def bench_batched(args):
    sc, specs, moving = build_batched(args)
    if args.schedule:
        sc.set_solver_config(**json.loads(args.schedule))
    sc.step(args.settle, stats=False)
    for e, b in enumerate(moving):
        sc.set_kinematic_bodies(e, b)
    sc.step(1)
    if not args.schedule and not args.no_autotune:
        sc.autotune(steps=2)
    sc.set_step_graphs(args.launch == "graphs")
    for _ in range(args.warmup):
        sc.step(1)
    device_sync()
    # stats of one step (synchronising), then the timed steps without host reads
    st = sc.step(1)
    cs_step = sum(x["contacts"] * x["sweeps"] for x in st)
    device_sync()
    t0 = time.perf_counter()
    sc.step(args.steps, stats=False)
    device_sync()
    wall = time.perf_counter() - t0
    # one eager step for the phase breakdown
    sc.set_step_graphs(False)
    st2 = sc.step(1)
    ph = sc.get_phase_times()
    n = sum(len(s["x"]) for s in specs)
    contacts = sum(x["contacts"] for x in st2)
    line = {
        "metric": "contacts*PGS-sweeps/s (whole step)",
        "value": cs_step * args.steps / wall,
        "unit": "contacts*sweeps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched: {len(specs)} independent beds, {n} spheres (log-uniform 500-20000 per "
                               f"bed), blade or bucket at U(0.3, 1.5) m/s, dt 1/60 s, {args.sweeps} sweeps, "
                               f"prev warm start, {'eager launches' if args.launch == 'eager' else 'step graphs'}",
                   "contacts_per_step": contacts, "steps_per_s": args.steps / wall,
                   "schedule": sc.get_solver_config(),
                   "eager_phase_ms": {k: float(v) for k, v in ph.items()}},
    }
    print(json.dumps(line), flush=True)


def bench_copy(args):
    """Calibration workload for the HBM traffic counters: device-to-device
    copies of a known size (the runtime's copy kernel), 256 MiB each."""
    from paper_2011_00459_amd.devmem import DeviceArray, hip
    nbytes = 256 << 20
    a, b = DeviceArray(nbytes // 4), DeviceArray(nbytes // 4)
    a.zero()
    h = hip()
    device_sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rc = h.hipMemcpy(ctypes.c_void_p(b.ptr), ctypes.c_void_p(a.ptr), nbytes, 3)
        if rc != 0:
            raise RuntimeError(f"hipMemcpy D2D failed ({rc})")
    device_sync()
    wall = time.perf_counter() - t0
    print(json.dumps({"workload": "copy", "bytes_per_copy": nbytes, "copies": args.steps,
                      "read_plus_write_GBps": 2 * nbytes * args.steps / wall / 1e9}), flush=True)


ADVECT_BYTES = 40  # per voxel: mf in (8), u in (24), mf out (8); neighbours' values are re-reads


def bench_voxels(args):
    """Mesoscale voxel step on a 256 x 256 x 128 dig-site grid (8.4 M voxels,
    l0 = 0.05 m), inputs resident in HBM: the cut of the resting solid under
    the zone wedges the particle step predicted for a blade, the conserved
    advection of the fluidized mass, the deposit of particle-free fluid outside
    the zone and the surface heights (Eq. surface).  The advection kernel's
    device time comes from HIP events on the library's stream (the default
    stream here); the coarse-graining of a 50,000-sphere bed is timed beside
    it."""
    import math
    from paper_2011_00459_amd.devmem import DeviceArray, hip
    h = hip()
    w = SG.voxel_workload(seed=11)
    vt = SG.voxel_terrain(seed=12)
    nx, ny, nz = w["dims"]
    nv = nx * ny * nz
    l0, org = w["l0"], w["origin"]
    # the terrain as the particle step's heightfield, a blade with a tool on it
    hf = dict(type="hfield", nx=nx, ny=ny, ox=org[0] + 0.5 * l0, oy=org[1] + 0.5 * l0, l0=l0,
              h=np.float32(vt["h"]).ravel())
    bodies = [dict(pos=(0, 0, 0), quat=(1, 0, 0, 0), linvel=(0, 0, 0), angvel=(0, 0, 0), shapes=[hf]),
              dict(pos=(0, 0, 0), quat=(1, 0, 0, 0), linvel=(1.0, 0, 0), angvel=(0, 0, 0),
                   shapes=[dict(type="box", half=(0.02, 3.0, 0.5), off=(4.0, 6.0, 3.5))])]
    tool = dict(body=1, n_wedges=8, edge0=(4.0, 3.0, 3.0), edge1=(4.0, 9.0, 3.0), n_c=(1, 0, 0),
                phi=math.radians(33), heap=0.1)
    top = nz * l0
    spec = dict(x=SG.fp32([[0.5, 0.5, top - 0.3]]), r=SG.fp32([0.2]), v=np.zeros((1, 3)), w=np.zeros((1, 3)),
                id=np.arange(1), bodies=bodies, tools=[tool], material=SG.material(0.5, 0.0), dt=w["dt"],
                gravity=(0.0, 0.0, 0.0), max_sweeps=0, tol=0.0, warm_start="cold", grid_lo=(0.0, 0.0, 0.0),
                grid_hi=(nx * l0, ny * l0, top), r_ref=0.05)
    sc = T.scene_from_specs(spec)
    sc.step(1)
    phi, wc = DeviceArray.from_host(vt["phi"], np.float64), DeviceArray.from_host(vt["wc"], np.float64)
    rho_p = DeviceArray.from_host(vt["rho_p"], np.float64)
    mf = [DeviceArray.from_host(vt["mf"] + w["mf"], np.float64), DeviceArray(w["mf"].shape, np.float64)]
    u = DeviceArray.from_host(w["u"], np.float64)
    hd = DeviceArray((ny, nx), np.float64)
    grid = (org, l0, w["dims"])
    # five events per timed step: around the cut, the advection, the deposit and the surface
    ev = []
    for _ in range(5 * (args.steps + 1)):
        e = ctypes.c_void_p()
        if h.hipEventCreate(ctypes.byref(e)) != 0:
            raise RuntimeError("hipEventCreate failed")
        ev.append(e)

    def meso_step(k, timed):
        a, b = mf[k % 2], mf[(k + 1) % 2]

        def mark(q):
            if timed is not None:
                h.hipEventRecord(ev[5 * timed + q], None)
        mark(0)
        sc.convert_cut(0, *grid, vt["rho_b"], phi.ptr, wc.ptr, a.ptr, wedges=None, sync=False)
        mark(1)
        sc.advect_fluid(*grid, w["dt"], u.ptr, a.ptr, b.ptr, sync=False)
        mark(2)
        sc.convert_deposit(0, *grid, vt["rho_b"], vt["w_dep"], rho_p.ptr, phi.ptr, wc.ptr, b.ptr, wedges=None,
                           sync=False)
        mark(3)
        sc.terrain_from_voxels(0, *grid, phi.ptr, hd.ptr)
        mark(4)

    m0 = float(np.sum(vt["phi"] * vt["wc"]) * vt["rho_b"] * l0 ** 3 + np.sum(vt["mf"] + w["mf"]))
    for k in range(args.warmup):
        meso_step(k, None)
    device_sync()
    t0 = time.perf_counter()
    for k in range(args.steps):
        meso_step(args.warmup + k, k)
    device_sync()
    wall = time.perf_counter() - t0
    op_ms = {"cut": 0.0, "advect": 0.0, "deposit": 0.0, "surface": 0.0}
    for k in range(args.steps):
        for q, name in enumerate(op_ms):
            ms = ctypes.c_float()
            h.hipEventElapsedTime(ctypes.byref(ms), ev[5 * k + q], ev[5 * k + q + 1])
            op_ms[name] += ms.value / args.steps
    dev_ms = op_ms["advect"] * args.steps
    last = mf[(args.warmup + args.steps) % 2].get()
    m1 = float(np.sum(phi.get() * wc.get()) * vt["rho_b"] * l0 ** 3 + np.sum(last))
    cfl = sc.advect_fluid(*grid, w["dt"], u.ptr, mf[0].ptr, mf[1].ptr)
    # coarse-graining of a settled-size bed onto its own grid, event-timed the same way
    bed = SG.bed_scene(seed=2, n=args.n, r0=0.03, spread=0.1, lx=4.0, ly=2.0, mu=0.7, c=2000.0, sweeps=50,
                       tool="none")
    bsc = T.scene_from_specs(bed, cap_contacts=16 * args.n)
    bsc.step(2)
    lo, l0c, dims_c = (-2.1, -1.1, -0.05), 0.06, (72, 38, 16)
    nvc = int(np.prod(dims_c))
    rho, mom, uc = DeviceArray((nvc,), np.float64), DeviceArray((nvc, 3), np.float64), DeviceArray((nvc, 3), np.float64)
    cg = {}
    for kern, R in (("heaviside", 0.0), ("gauss", 0.06)):
        bsc.coarse_grain(0, lo, l0c, dims_c, rho.ptr, mom.ptr, uc.ptr, kernel=kern, R=R)
        device_sync()
        h.hipEventRecord(ev[0], None)
        for _ in range(10):
            bsc.coarse_grain(0, lo, l0c, dims_c, rho.ptr, mom.ptr, uc.ptr, kernel=kern, R=R)
        h.hipEventRecord(ev[1], None)
        h.hipEventSynchronize(ev[1])
        ms = ctypes.c_float()
        h.hipEventElapsedTime(ctypes.byref(ms), ev[0], ev[1])
        cg[kern] = dict(ms=ms.value / 10, particles=args.n, voxels=nvc)
    adv_ms = dev_ms / args.steps
    achieved = ADVECT_BYTES * nv / (adv_ms * 1e-3) / 1e9
    line = {
        "metric": "voxel updates/s (mesoscale step)", "value": nv * args.steps / wall, "unit": "voxels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "mesoscale dig site: 256x256x128 voxels l0 0.05 m, rolling terrain, a blade's "
                               "8-wedge zone cutting 0.3-1.5 m deep, fluidized soil in an ellipsoidal zone, swirl "
                               "velocity at Courant <= 0.4, dt 1/60 s: cut + advection + deposit + surface",
                   "courant": cfl, "advect_device_ms": adv_ms, "op_device_ms": op_ms,
                   "mass_drift_rel": abs(m1 - m0) / m0,
                   "coarse_grain_bed": cg},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": source_traffic(ADVECT_TRAFFIC, "terrain_voxels.hip"),
                     "algorithmic_bytes_per_launch": ADVECT_BYTES * nv, "kernel": "k_advect"},
    }
    if not args.no_cpu:
        sys.path.insert(0, os.path.join(ROOT, "oracle"))
        import pyoracle as O
        # the oracle's own wedges for the same tool on the same terrain, then
        # its mesoscale step (cut, advection, deposit, surface) on the same grid
        ow = O.predict_wedges(tool, bodies)
        ophi, owc, omf = vt["phi"], vt["wc"], vt["mf"] + w["mf"]
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < min(args.cpu_seconds, 15.0):
            ophi, omf, _ = O.convert_cut(ophi, owc, omf, ow, *grid, vt["rho_b"])
            omf, _ = O.advect(omf, w["u"], *grid, w["dt"])
            ophi, owc, omf, _ = O.convert_deposit(ophi, owc, omf, vt["rho_p"], ow, *grid, vt["rho_b"], vt["w_dep"])
            O.surface_heights(ophi, *grid)
            reps += 1
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": nv * reps / dt, "unit": "voxels/s", "cores": 1, "kind": "oracle",
                                "sample": f"{reps} oracle mesoscale steps (cut, advection, deposit, surface) of the "
                                          "same 8.4 M-voxel grid"}
    print(json.dumps(line), flush=True)


def mlp_throughput(n=1 << 22):
    """The learned-start network on MFMA (BF16 inference) and the FP32
    training kernels: device time per call from HIP events, TFLOP/s."""
    from paper_2011_00459_amd import learn as LN
    from paper_2011_00459_amd.devmem import DeviceArray
    rng = np.random.default_rng(0)
    w = LN.flatten(LN.init_weights(0))
    W = DeviceArray.from_host(w)
    F = DeviceArray.from_host(rng.normal(0, 1, (n, 12)).astype(np.float32))
    Y = DeviceArray((n, 3))
    out = {}
    flops_fwd = 2 * (12 * 64 + 64 * 64 + 64 * 3)
    for name, bf16 in (("bf16_mfma_forward", True), ("fp32_forward", False)):
        T.mlp_forward(W.ptr, F.ptr, n, Y.ptr, bf16=bf16)
        device_sync()
        t0 = time.perf_counter()
        for _ in range(20):
            T.mlp_forward(W.ptr, F.ptr, n, Y.ptr, bf16=bf16)
        device_sync()
        dt = (time.perf_counter() - t0) / 20
        tf = flops_fwd * n / dt / 1e12
        peak = 2500.0 if bf16 else 157.3
        out[name] = dict(samples=n, ms=1e3 * dt, tflops=tf, peak_tflops=peak, frac=tf / peak)
    B = 1 << 16
    ns = T.mlp_grad_scratch_floats(B)
    G, L, S = DeviceArray(T.MLP_TRAINABLE), DeviceArray(1), DeviceArray(ns)
    lab = DeviceArray.from_host(rng.normal(0, 1, (B, 3)).astype(np.float32))
    T.mlp_loss_grad(W.ptr, F.ptr, lab.ptr, B, G.ptr, L.ptr, S.ptr, ns)
    device_sync()
    t0 = time.perf_counter()
    for _ in range(10):
        T.mlp_loss_grad(W.ptr, F.ptr, lab.ptr, B, G.ptr, L.ptr, S.ptr, ns)
    device_sync()
    dt = (time.perf_counter() - t0) / 10
    tf = 3 * flops_fwd * B / dt / 1e12  # forward + backward ~ 3x the forward
    out["fp32_train_step"] = dict(samples=B, ms=1e3 * dt, tflops=tf, peak_tflops=157.3, frac=tf / 157.3)
    return out


def learned_eval(args):
    """Train the learned start on the GPU (column trajectories of the plain
    solver) and measure steps/s and sweeps to R_k <= 1e-4 with the cold,
    previous-step and learned starts, each from one shared settled state."""
    from paper_2011_00459_amd import learn as LN
    t0 = time.perf_counter()
    feat, label = LN.gen_dataset(n_envs=16, steps=120, cap=1_000_000, seed=100)
    tr = LN.Trainer(LN.init_weights(0, LN.input_scale(feat)), feat, LN.residual_targets(feat, label), batch=4096)
    hist = tr.fit(epochs=20, lr=3e-3, lr_end=2e-4)
    w = tr.weights()
    train_s = time.perf_counter() - t0
    res = {"training": dict(samples=len(feat), epochs=20, loss_first=hist[0], loss_last=hist[-1],
                            seconds=train_s)}
    cols = LN.column_batch(8, seed=900)
    res["columns_1000"] = LN.sweeps_to_tol(cols, weights=w, settle=60, steps=10, tol=1e-4, max_sweeps=4000)
    specs = SG.batch_specs(seed=3000, n_envs=args.eval_envs, sweeps=100)
    mat = specs[0]["material"]
    specs = [dict(s, material=mat) for s in specs]
    res[f"batched_{args.eval_envs}"] = LN.sweeps_to_tol(specs, weights=w, settle=40, steps=4, tol=1e-4,
                                                       max_sweeps=3000)
    for k in ("columns_1000", f"batched_{args.eval_envs}"):
        r = res[k]
        r["learned_vs_cold_steps_per_s"] = r["learned"]["steps_per_s"] / r["cold"]["steps_per_s"]
        r["learned_vs_prev_steps_per_s"] = r["learned"]["steps_per_s"] / r["prev"]["steps_per_s"]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=50000)
    ap.add_argument("--sweeps", type=int, default=None, help="PGS sweeps (150 for the bed, 100 batched)")
    ap.add_argument("--settle", type=int, default=150)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=("bed", "batched", "copy", "mlp", "voxels"), default="bed",
                    help="mlp: the learned-start network's throughput alone (one JSON line); voxels: the "
                         "mesoscale advection step")
    ap.add_argument("--envs", type=int, default=256)
    ap.add_argument("--schedule", default="", help="PGS schedule as JSON (set_solver_config fields)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-start training and evaluation")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default PGS schedule")
    ap.add_argument("--launch", choices=("eager", "graphs"), default="eager",
                    help="launch every kernel of a step (measured faster here) or replay step graphs")
    ap.add_argument("--eval-envs", type=int, default=64, help="batched beds of the warm-start evaluation")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is design-only",
              file=sys.stderr)
        sys.exit(2)
    if args.sweeps is None:
        args.sweeps = 100 if args.workload == "batched" else 150
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "copy":
        bench_copy(args)
        return
    if args.workload == "voxels":
        bench_voxels(args)
        return
    if args.workload == "mlp":
        print(json.dumps({"workload": "learned-start network, 4,194,304 contacts", "mlp": mlp_throughput()}))
        return

    sc, spec, blade, est_top = build_bed(args)
    if args.schedule:
        sc.set_solver_config(**json.loads(args.schedule))
    st0, top = settle(sc, spec, blade, args.settle)
    print(f"# settled: {st0['contacts']} contacts, top {top:.3f} m (estimate {est_top:.3f})", file=sys.stderr,
          flush=True)
    moving = dict(blade)
    moving["pos"] = (-1.6, 0.0, top - 0.2 + 0.3)
    moving["linvel"] = (1.0, 0.0, 0.0)
    bodies = [dict(spec["bodies"][0], id=0), dict(moving, id=1)]
    sc.set_kinematic_bodies(0, bodies)
    tuned = None
    if not args.schedule and not args.no_autotune:
        tuned = sc.autotune(steps=3)  # times the candidate schedules from this state, then restores it
        sc.set_step_graphs(args.launch == "graphs")
    for _ in range(args.warmup):
        sc.step(1)
    wall, tot_cs, pgs_bytes, pgs_ms, stats = timed_steps(sc, args.steps)
    value = tot_cs / wall
    ms_per_step = 1e3 * wall / args.steps
    pgs_launch_ms = pgs_ms / args.steps
    achieved = pgs_bytes / args.steps / (pgs_launch_ms * 1e-3) / 1e9 if pgs_launch_ms > 0 else 0.0
    last = stats[-1][0]
    phases = {k: float(np.mean([ph[k] for _, ph in stats])) for k in ("detect", "rows", "pgs", "finish", "step")}
    f, _ = sc.get_contact_forces(0, 1)
    aggs = sc.get_aggregates(0)
    line = {
        "metric": "contacts*PGS-sweeps/s (whole step)",
        "value": value,
        "unit": "contacts*sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"bulldozing bed: {args.n} spheres r 0.03 m, 4x2 m, box blade 1.5x0.05x0.6 m "
                               f"at 1 m/s, 0.2 m deep, dt 1/60 s, {args.sweeps} sweeps, prev warm start",
                   "contacts_per_step": last["contacts"], "pair_contacts": last["pair_contacts"],
                   "colours": last["colours"], "sweeps": last["sweeps"],
                   "pgs_ms_per_step": pgs_launch_ms,
                   "schedule": sc.get_solver_config(), "autotune_ms_per_step": tuned[1] if tuned else None,
                   "phase_ms": phases,
                   "blade_force_x_N": float(f[0])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": pgs_traffic(),
                     "algorithmic_bytes_per_launch": pgs_bytes / args.steps,
                     "kernel": "k_pgs (persistent colour-synchronous PGS)"},
    }
    if not args.no_learned:
        line["mlp"] = mlp_throughput()
        line["warm_start_to_1e-4"] = learned_eval(args)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
