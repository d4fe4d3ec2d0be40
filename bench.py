#!/usr/bin/env python3
"""Benchmark of the agitated-soil particle step on one MI355X.

One step = detection, canonical order, rows, colouring, warm start, PGS,
integration, body forces and zone aggregates, every phase on the GPU.  Inputs
are resident in HBM when the timed region starts.

Default line (the headline): 256 independent beds stepped together, particle
counts log-uniform in [500, 20000] (1.21 M spheres, about 3.2 M contacts),
each a 3 x 2 m bed with a blade or an open bucket on a random heading at
U(0.3, 1.5) m/s, dt 1/60 s, 100 PGS sweeps, previous-step warm start, settled
on the GPU before timing.  value = sum over the timed steps of contacts x PGS
sweeps / wall time of those steps.

roofline: the per-env PGS kernel (k_pgs_env): algorithmic bytes (176 B per
pair contact-sweep, 128 B per boundary contact-sweep) / its HIP-event
duration on the scene's stream, summed over the timed steps.
cpu_baseline: the FP64 oracle as it stands on the same 256 beds (settled by
the oracle itself), one process per host core, one step of each bed.

Extra keys: the 50,000-sphere bulldozing bed (bed50k), the 500,000-sphere
excavation with a bucket on a dig path (excavation500k), the network's
throughput (mlp) and the sweeps / steps per second to R_k <= 1e-4 of the
cold, previous-step and learned starts on the 256 beds (warm_start_to_1e-4).
"""
import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2011_00459_amd import scenegen as SG  # noqa: E402
from paper_2011_00459_amd import terrain as T  # noqa: E402
from paper_2011_00459_amd import zones as Z  # noqa: E402

HBM_PEAK_GBS = 8000.0
PAIR_BYTES, BOUND_BYTES = 176, 128

# HBM traffic of one PGS launch, from the FETCH_SIZE and WRITE_SIZE counter
# runs scaled by a copy kernel of known size (profiles named below); valid
# only for the kernel source it was measured on, else reported as null.
PGS_TRAFFIC = {
    "batched": {"kernels_sha256_prefix": "02315f89cb19c419", "bytes_per_launch": 52.76e9,
                "profile": "profiles/k_pgs_env_batched256_hbm_traffic.md"},
    "bed": {"kernels_sha256_prefix": "02315f89cb19c419", "bytes_per_launch": 3.494e9,
            "profile": "profiles/k_pgs_bed50k_hbm_traffic.md"},
    "excavation": {"kernels_sha256_prefix": "02315f89cb19c419", "bytes_per_launch": 71.00e9,
                   "profile": "profiles/k_pgs_excavation500k_hbm_traffic.md"},
}
# The same for k_advect on the 256 x 256 x 128 voxel grid
# (profiles/k_advect_voxels256_kernel_trace.md), keyed to terrain_voxels.hip.
ADVECT_TRAFFIC = {"kernels_sha256_prefix": "92ca9f936e1a6af0", "bytes_per_launch": 0.3757e9,
                  "profile": "profiles/k_advect_voxels256_kernel_trace.md"}


def source_traffic(entry, source="terrain_kernels.hip"):
    import hashlib
    if entry.get("bytes_per_launch") is None:
        return None
    with open(os.path.join(ROOT, "paper_2011_00459_amd", "csrc", source), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return entry["bytes_per_launch"] if sha == entry["kernels_sha256_prefix"] else None


def device_sync():
    hip = ctypes.CDLL("libamdhip64.so.7")
    rc = hip.hipDeviceSynchronize()
    if rc != 0:
        raise RuntimeError(f"hipDeviceSynchronize failed ({rc})")


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def timed_steps(sc, k):
    """k steps, one call each (every call waits for its step and returns its
    statistics): contacts x sweeps, the PGS's algorithmic bytes and its
    HIP-event time per step, summed."""
    device_sync()
    t0 = time.perf_counter()
    tot = dict(cs=0, bytes=0, pgs_ms=0.0, contacts=0, pairs=0, steps=0)
    last = None
    for _ in range(k):
        st = sc.step(1)
        ph = sc.get_phase_times()
        for x in st:
            tot["cs"] += x["contacts"] * x["sweeps"]
            tot["bytes"] += (x["pair_contacts"] * PAIR_BYTES + (x["contacts"] - x["pair_contacts"]) * BOUND_BYTES) \
                * x["sweeps"]
        tot["pgs_ms"] += ph["pgs"]
        tot["steps"] += 1
        last = (st, ph)
    device_sync()
    tot["wall"] = time.perf_counter() - t0
    tot["last"] = last
    return tot


def phase_ms(ph):
    # phases a step-graph replay does not time are reported as null
    return {k: None if math.isnan(v) else float(v) for k, v in ph.items()}


def roofline(tot, kernel, traffic_key):
    ms = tot["pgs_ms"] / tot["steps"]
    bpl = tot["bytes"] / tot["steps"]
    if math.isnan(ms):
        # a step-graph replay is timed only as a whole
        return {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
                "traffic": source_traffic(PGS_TRAFFIC[traffic_key]), "algorithmic_bytes_per_launch": bpl,
                "launch_ms": None, "kernel": kernel, "note": "step graphs: the PGS launch is not timed alone; "
                "use --launch eager"}
    achieved = bpl / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": source_traffic(PGS_TRAFFIC[traffic_key]),
            "algorithmic_bytes_per_launch": bpl, "launch_ms": ms, "kernel": kernel}


def pgs_kernel_name(sc):
    mode = sc.get_solver_config()["mode"]
    return {"grouped": "k_pgs (grouped persistent colour-synchronous PGS)",
            "spread": "k_pgs (spread: one env on all XCDs, colour-synchronous PGS)",
            "per_env": "k_pgs_env (per-env persistent colour-synchronous PGS)"}[mode]


# bulk properties of the aggregate in the timed macroscale step: the bed's
# friction (tan phi_b = 0.7) and cohesion (2 kPa), a stiff bulk
MACRO_PARAMS = dict(E_b=1e7, c_b=2000.0, mu_ab=0.4, mu_ac=0.7, cas_ab=1.0, cas_ac=0.001)


def time_macro(sc, env=0, calls=10, equipment=None):
    """Wall time of the macroscale step of env's zones on the state after the
    timed steps (each call synchronises), and what it found."""
    res = sc.macro_step(env, equipment=equipment, **MACRO_PARAMS)
    t0 = time.perf_counter()
    for _ in range(calls):
        res = sc.macro_step(env, equipment=equipment, **MACRO_PARAMS)
    ms = 1e3 * (time.perf_counter() - t0) / calls
    if not res:
        return dict(ms_per_call=ms, zones=0)
    o = res[0]
    out = dict(ms_per_call=ms, zones=len(res), n_cand=[int(k) for k in o["n_cand"]], n_points=list(o["n_points"]),
               iterations=int(o["sweeps"]), aggregate_mass_kg=float(o["M"]), v_after=[float(k) for k in o["v"]],
               force_on_tool_N=[float(k) for k in o["force"]])
    if equipment:
        out.update(tool_v_after=[float(k) for k in o["v_b"]], drive_impulse=[float(k) for k in o["lam_drive"]])
    return out


def bucket_equipment(body_id, speed):
    """The excavation's 1.2 x 1.0 x 0.8 m bucket as a dynamic body: 1.5 t, a
    box's inertia, driven at its dig speed with 60 kN and 20 kN m limits."""
    m, a, b, c = 1500.0, 1.0, 1.2, 0.8
    inertia = (m * (b * b + c * c) / 12.0, m * (a * a + c * c) / 12.0, m * (a * a + b * b) / 12.0, 0.0, 0.0, 0.0)
    return [dict(body=body_id, mass=m, inertia=inertia, v_target=(speed, 0.0, 0.0), w_target=(0.0, 0.0, 0.0),
                 f_max=6e4, t_max=2e4, gamma_drive=1e-6)]


# ---------------------------------------------------------------------------
# config 3: 256 batched beds (the headline)
# ---------------------------------------------------------------------------
def build_batched(args, n_envs=None, sweeps=None):
    specs = SG.batch_specs(seed=3000, n_envs=n_envs or args.envs, sweeps=sweeps or args.sweeps)
    mat = specs[0]["material"]
    specs = [dict(s, material=mat, warm_start="prev") for s in specs]
    nmax = max(len(s["x"]) for s in specs)
    sc = T.scene_from_specs(specs, cap_particles=nmax, cap_contacts=8 * nmax)
    # the tools are held still while the beds settle
    moving = []
    for e, s in enumerate(specs):
        b = [dict(x, id=i) for i, x in enumerate(s["bodies"])]
        moving.append([dict(x) for x in b])
        for x in b:
            x["linvel"] = (0.0, 0.0, 0.0)
        sc.set_kinematic_bodies(e, b)
    return sc, specs, moving


def leg_batched(args):
    sc, specs, moving = build_batched(args)
    if args.schedule:
        sc.set_solver_config(**json.loads(args.schedule))
    sc.step(args.settle, stats=False)
    for e, b in enumerate(moving):
        sc.set_kinematic_bodies(e, b)
    sc.step(1)
    tuned = None
    if not args.schedule and not args.no_autotune:
        tuned = sc.autotune(steps=2)
    sc.set_step_graphs(args.launch == "graphs")
    sc.step(args.warmup, stats=False)
    tot = timed_steps(sc, args.steps)
    st, ph = tot["last"]
    n = sum(len(s["x"]) for s in specs)
    out = dict(value=tot["cs"] / tot["wall"], ms_per_step=1e3 * tot["wall"] / args.steps,
               steps_per_s=args.steps / tot["wall"], spheres=n, envs=len(specs),
               contacts_per_step=sum(x["contacts"] for x in st), colours_max=max(x["colours"] for x in st),
               sweeps=st[0]["sweeps"], schedule=sc.get_solver_config(),
               autotune_ms_per_step=tuned[1] if tuned else None,
               phase_ms_last_step=phase_ms(ph),
               roofline=roofline(tot, pgs_kernel_name(sc), "batched"))
    sc.close()
    return out, specs


# ---------------------------------------------------------------------------
# config 2: the 50,000-sphere bulldozing bed
# ---------------------------------------------------------------------------
def leg_bed(args, n=50000, sweeps=150):
    spec = SG.bed_scene(seed=2, n=n, r0=0.03, spread=0.1, lx=4.0, ly=2.0, mu=0.7, c=2000.0, sweeps=sweeps,
                        tool="none")
    solids = float(np.sum(4.0 / 3.0 * np.pi * spec["r"] ** 3))
    est_top = solids / (4.0 * 2.0 * 0.6)
    blade = SG.box_blade(-1.6, est_top - 0.2, width=1.5, thick=0.05, height=0.6, vx=0.0)
    spec["bodies"] = spec["bodies"] + [blade]
    spec["warm_start"] = "prev"
    sc = T.scene_from_specs(spec, cap_contacts=16 * n)
    if args.schedule:
        sc.set_solver_config(**json.loads(args.schedule))
    sc.step(args.settle, stats=False)
    p = sc.get_particles(0)
    top = float(np.percentile(p["x"][:, 2] + p["r"], 99.0))
    # the blade 0.2 m below the settled surface, cutting along +x at 1 m/s,
    # with its active zone (Eq. failure_plane wedge) aggregated every step
    moving = dict(blade, pos=(-1.6, 0.0, top - 0.2 + 0.3), linvel=(1.0, 0.0, 0.0))
    moving["zone_planes"] = Z.blade_zone(moving, 0.7, top)
    sc.set_kinematic_bodies(0, [dict(spec["bodies"][0], id=0), dict(moving, id=1)])
    tuned = None
    if not args.schedule and not args.no_autotune:
        tuned = sc.autotune(steps=3)
    sc.set_step_graphs(args.launch == "graphs")
    sc.step(args.warmup, stats=False)
    tot = timed_steps(sc, args.steps)
    st, ph = tot["last"]
    f, _ = sc.get_contact_forces(0, 1)
    agg = sc.get_aggregates(0)
    out = dict(value=tot["cs"] / tot["wall"], ms_per_step=1e3 * tot["wall"] / args.steps, spheres=n,
               contacts_per_step=st[0]["contacts"], pair_contacts=st[0]["pair_contacts"],
               colours=st[0]["colours"], sweeps=st[0]["sweeps"], settled_top_m=top,
               schedule=sc.get_solver_config(), autotune_ms_per_step=tuned[1] if tuned else None,
               phase_ms_last_step=phase_ms(ph), blade_force_N=[float(x) for x in f],
               zone_particles=int(agg[0]["n_particles"]) if agg else 0,
               zone_mass_kg=float(agg[0]["M"]) if agg else 0.0,
               macro_step=time_macro(sc),
               roofline=roofline(tot, pgs_kernel_name(sc), "bed"))
    sc.close()
    return out


# ---------------------------------------------------------------------------
# config 5: the 500,000-sphere excavation with a bucket on a dig path
# ---------------------------------------------------------------------------
def leg_excavation(args, weights=None, n=500000, sweeps=200):
    spec = SG.excavation_scene(seed=5, n=n, sweeps=sweeps)
    floor, bucket = spec["bodies"][0], spec["bodies"][1]
    lattice_top = float(spec["grid_hi"][2]) - 0.5
    # settle with the bucket parked above the poured spheres
    parked = dict(bucket, pos=(-3.0, 0.0, lattice_top + 0.5), linvel=(0.0, 0.0, 0.0))
    spec = dict(spec, bodies=[floor, parked], warm_start="prev")
    sc = T.scene_from_specs(spec, cap_contacts=8 * n)
    if args.schedule:
        sc.set_solver_config(**json.loads(args.schedule))
    t0 = time.perf_counter()
    sc.step(args.settle_excavation, stats=False)
    settle_s = time.perf_counter() - t0
    p = sc.get_particles(0)
    top = float(np.percentile(p["x"][:, 2] + p["r"], 99.0))
    # dig path at 0.8 m/s: descend at 30 degrees until the bucket's bottom is
    # 0.4 m below the surface, then drag along +x (the timed steps), as the
    # excavation test of the paper digs with a bucket
    hh = 0.4  # half height of the 0.8 m bucket
    depth, speed = 0.4, 0.8
    start_bottom = top + 0.05
    descend = dict(parked, id=1, pos=(-3.0, 0.0, start_bottom + hh),
                   linvel=(speed * math.cos(math.radians(30)), 0.0, -speed * math.sin(math.radians(30))))
    zone = Z.wedge_planes(0.5, -hh, 1.2, top - (start_bottom + hh) + 0.3, Z.friction_angle(0.7))
    descend["zone_planes"] = zone
    drag = dict(descend, linvel=(speed, 0.0, 0.0))
    n_desc = int(round((0.05 + depth) / (speed * math.sin(math.radians(30))) / spec["dt"]))
    sc.set_kinematic_bodies(0, [dict(floor, id=0), descend])
    sc.step(1)
    if weights is not None:
        sc.set_mlp_weights(weights)
        sc.set_learned_precision(True)
        sc.set_warm_start("learned")
    sc.step(n_desc - 1, stats=False)
    # drag: the bucket keeps the pose the descent reached
    pose_z = start_bottom + hh - n_desc * spec["dt"] * speed * math.sin(math.radians(30))
    pose_x = -3.0 + n_desc * spec["dt"] * speed * math.cos(math.radians(30))
    drag = dict(drag, pos=(pose_x, 0.0, pose_z))
    drag["zone_planes"] = Z.wedge_planes(0.5, -hh, 1.2, top - pose_z + 0.3, Z.friction_angle(0.7))
    sc.set_kinematic_bodies(0, [dict(floor, id=0), drag])
    tuned = None
    if not args.schedule and not args.no_autotune:
        tuned = sc.autotune(steps=2)
    sc.set_step_graphs(args.launch == "graphs")
    sc.step(args.warmup, stats=False)
    tot = timed_steps(sc, args.steps)
    st, ph = tot["last"]
    f, _ = sc.get_contact_forces(0, 1)
    agg = sc.get_aggregates(0)
    out = dict(value=tot["cs"] / tot["wall"], ms_per_step=1e3 * tot["wall"] / args.steps, spheres=n,
               contacts_per_step=st[0]["contacts"], pair_contacts=st[0]["pair_contacts"],
               colours=st[0]["colours"], sweeps=st[0]["sweeps"], settled_top_m=top,
               settle_steps=args.settle_excavation, settle_s=settle_s, descent_steps=n_desc,
               warm_start="learned" if weights is not None else "prev",
               learned_fallback_last_step=int(st[0]["fallback_used"]),
               schedule=sc.get_solver_config(), autotune_ms_per_step=tuned[1] if tuned else None,
               phase_ms_last_step=phase_ms(ph), bucket_force_N=[float(x) for x in f],
               zone_particles=int(agg[0]["n_particles"]) if agg else 0,
               zone_mass_kg=float(agg[0]["M"]) if agg else 0.0,
               macro_step=time_macro(sc),
               macro_step_driven_bucket=time_macro(sc, equipment=bucket_equipment(1, speed)),
               roofline=roofline(tot, pgs_kernel_name(sc), "excavation"))
    sc.close()
    return out


# ---------------------------------------------------------------------------
# the oracle on the host cores: the same 256 beds, one process per core
# ---------------------------------------------------------------------------
def _oracle_settle(job):
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import pyoracle as O
    e, n_envs, settle, sweeps = job
    spec = SG.batch_spec(3000, e, sweeps=sweeps)
    spec = dict(spec, warm_start="prev", max_sweeps=10)
    o = O.OracleScene(spec)
    for _ in range(settle):
        o.step()
    return e, o.x, o.v, o.w, o.prev_keys, o.prev_lam


def _oracle_step(job):
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import pyoracle as O
    e, n_envs, sweeps, x, v, w, pk, pl = job
    spec = SG.batch_spec(3000, e, sweeps=sweeps)
    spec = dict(spec, x=x, v=v, w=w, warm_start="prev", max_sweeps=sweeps)
    o = O.OracleScene(spec)
    o.prev_keys, o.prev_lam = pk, pl
    t0 = time.perf_counter()
    out = o.step()
    return e, out["contacts"] * out["sweeps"], time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_batched(args):
    from multiprocessing import get_context
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    n_envs = args.envs
    specs = SG.batch_specs(seed=3000, n_envs=n_envs, sweeps=args.sweeps)
    order = sorted(range(n_envs), key=lambda e: -len(specs[e]["x"]))  # largest first
    del specs
    with get_context("fork").Pool(cores) as pool:
        settled = pool.map(_oracle_settle, [(e, n_envs, args.cpu_settle, args.sweeps) for e in order], chunksize=1)
        jobs = [(e, n_envs, args.sweeps, x, v, w, pk, pl) for e, x, v, w, pk, pl in settled]
        t0 = time.perf_counter()
        res = pool.map(_oracle_step, jobs, chunksize=1)
        wall = time.perf_counter() - t0
    cs = sum(r[1] for r in res)
    return dict(value=cs / wall, unit="contacts*sweeps/s", cores=cores, kind="oracle",
                nproc=os.cpu_count(), cpu_model=cpu_model(),
                sample=f"one FP64 oracle step ({args.sweeps} sweeps, previous-step start) of each of the same "
                       f"{n_envs} beds, settled by the oracle for {args.cpu_settle} steps of 10 sweeps first "
                       f"(untimed); {cores} worker processes, one bed at a time each, largest first; "
                       f"{cs:.3e} contact-sweeps in {wall:.1f} s wall ({sum(r[2] for r in res):.1f} s of CPU)")


# ---------------------------------------------------------------------------
# learned warm start: training on the GPU, then sweeps to R_k <= 1e-4
# ---------------------------------------------------------------------------
def learned_eval(args):
    from paper_2011_00459_amd import learn as LN
    t0 = time.perf_counter()
    feat, label = LN.gen_mixed_dataset(seed=100, cap=args.train_samples)
    tr = LN.Trainer(LN.init_weights(0, LN.input_scale(feat)), feat, LN.residual_targets(feat, label), batch=4096)
    hist = tr.fit(epochs=args.epochs, lr=1e-3, lr_end=1e-4)
    w = tr.weights()
    res = {"training": dict(samples=len(feat), epochs=args.epochs, loss_first=hist[0], loss_last=hist[-1],
                            seconds=time.perf_counter() - t0)}
    specs = SG.batch_specs(seed=3000, n_envs=args.envs, sweeps=100)
    mat = specs[0]["material"]
    specs = [dict(s, material=mat) for s in specs]
    r = LN.sweeps_to_tol(specs, weights=w, settle=args.settle, steps=args.eval_steps, tol=1e-4,
                         max_sweeps=5000, graphs=False)
    r["learned_vs_cold_steps_per_s"] = r["learned"]["steps_per_s"] / r["cold"]["steps_per_s"]
    r["learned_vs_prev_steps_per_s"] = r["learned"]["steps_per_s"] / r["prev"]["steps_per_s"]
    r["prev_vs_cold_steps_per_s"] = r["prev"]["steps_per_s"] / r["cold"]["steps_per_s"]
    res[f"batched_{args.envs}"] = r
    cols = LN.column_batch(8, seed=900)
    c = LN.sweeps_to_tol(cols, weights=w, settle=60, steps=10, tol=1e-4, max_sweeps=5000)
    c["learned_vs_cold_steps_per_s"] = c["learned"]["steps_per_s"] / c["cold"]["steps_per_s"]
    c["learned_vs_prev_steps_per_s"] = c["learned"]["steps_per_s"] / c["prev"]["steps_per_s"]
    c["prev_vs_cold_steps_per_s"] = c["prev"]["steps_per_s"] / c["cold"]["steps_per_s"]
    res["columns_1000"] = c
    return res, w


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




def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=("batched", "bed", "excavation", "copy", "mlp", "voxels"),
                    default="batched",
                    help="batched: the headline line (256 beds) with the other workloads as extra keys; bed, "
                         "excavation: that workload alone; mlp: the network's throughput; voxels: the "
                         "mesoscale step; copy: the traffic-counter calibration")
    ap.add_argument("--envs", type=int, default=256)
    ap.add_argument("--sweeps", type=int, default=100, help="PGS sweeps of the batched beds")
    ap.add_argument("--settle", type=int, default=150, help="settling steps of the beds before timing")
    ap.add_argument("--settle-excavation", type=int, default=120)
    ap.add_argument("--n", type=int, default=50000, help="spheres of the bulldozing bed (voxels workload too)")
    ap.add_argument("--cpu-settle", type=int, default=30, help="oracle settling steps of each bed (untimed)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline only: no bed, excavation, mlp, warm start")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-start training and evaluation")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default PGS schedule")
    ap.add_argument("--schedule", default="", help="PGS schedule as JSON (set_solver_config fields)")
    ap.add_argument("--launch", choices=("eager", "graphs"), default="eager",
                    help="launch every kernel of a step (measured faster here) or replay step graphs")
    ap.add_argument("--train-samples", type=int, default=2_000_000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--eval-steps", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is design-only",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "copy":
        bench_copy(args)
        return
    if args.workload == "voxels":
        bench_voxels(args)
        return
    if args.workload == "mlp":
        print(json.dumps({"workload": "learned-start network, 4,194,304 contacts", "mlp": mlp_throughput()}))
        return
    base = {"metric": "contacts*PGS-sweeps/s (whole step)", "unit": "contacts*sweeps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic"}
    if args.workload == "bed":
        r = leg_bed(args, n=args.n)
        line = dict(base, value=r.pop("value"), ms_per_step=r.pop("ms_per_step"), roofline=r.pop("roofline"),
                    config={"workload": f"bulldozing bed: {args.n} spheres r 0.03 m, 4x2 m, box blade "
                                        "1.5x0.05x0.6 m at 1 m/s, 0.2 m deep, dt 1/60 s, 150 sweeps, prev warm "
                                        "start, active zone aggregated every step", **r})
        print(json.dumps(line), flush=True)
        return
    if args.workload == "excavation":
        r = leg_excavation(args)
        line = dict(base, value=r.pop("value"), ms_per_step=r.pop("ms_per_step"), roofline=r.pop("roofline"),
                    config={"workload": "excavation: 500000 spheres r 0.02 m U(0.85, 1.15), 8x4 m bed, open bucket "
                                        "1.2x1.0x0.8 m dragged at 0.8 m/s 0.4 m deep after a 30-degree descent, "
                                        "dt 1/60 s, 200 sweeps, active zone aggregated every step", **r})
        print(json.dumps(line), flush=True)
        return

    log("batched beds")
    r, _ = leg_batched(args)
    line = dict(base, value=r.pop("value"), ms_per_step=r.pop("ms_per_step"), roofline=r.pop("roofline"))
    line["config"] = {"workload": f"batched: {r['envs']} independent beds, {r['spheres']} spheres (log-uniform "
                                  "500-20000 per bed), blade or bucket at U(0.3, 1.5) m/s, dt 1/60 s, "
                                  f"{args.sweeps} sweeps, prev warm start, "
                                  f"{'eager launches' if args.launch == 'eager' else 'step graphs'}", **r}
    weights = None

    def extra(key, fn, *a, **kw):
        # an extra workload that fails records its error; the headline stands
        log(key)
        t0 = time.perf_counter()
        try:
            out = fn(*a, **kw)
        except Exception as e:  # noqa: BLE001
            line[key] = {"error": f"{type(e).__name__}: {e}"}
            out = None
        log(f"{key}: {time.perf_counter() - t0:.1f} s")
        return out

    if not args.no_extras:
        r = extra("mlp", mlp_throughput)
        if r is not None:
            line["mlp"] = r
        if not args.no_learned:
            r = extra("warm_start_to_1e-4", learned_eval, args)
            if r is not None:
                line["warm_start_to_1e-4"], weights = r
        r = extra("bed50k", leg_bed, args)
        if r is not None:
            line["bed50k"] = r
        r = extra("excavation500k", leg_excavation, args, weights=weights)
        if r is not None:
            line["excavation500k"] = r
    if not args.no_cpu:
        r = extra("cpu_baseline", cpu_baseline_batched, args)
        if r is not None:
            line["cpu_baseline"] = r
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
