"""PyTorch as the library's device memory and streams.

A child process imports PyTorch before the library (paper_2011_00459_amd.
terrain.torch_first), so the library binds to the HIP runtime the PyTorch
wheel carries.  There, a scene runs on a torch.cuda.Stream with its buffers
from PyTorch's caching allocator, and the network kernel reads and writes
torch tensors; every result must equal, bit for bit, the same work done in
this process on the library's own runtime (hipMalloc, the null stream)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2011_00459_amd import scenegen as SG

pytestmark = pytest.mark.gpu

T = pytest.importorskip("paper_2011_00459_amd.terrain")
D = pytest.importorskip("paper_2011_00459_amd.devmem")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_2011_00459_amd import terrain as T
torch = T.torch_first()
from paper_2011_00459_amd import scenegen as SG
cfg = json.loads(sys.argv[3])
T.lib()
maps = open("/proc/self/maps").read()
runtimes = sorted({l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l})
print("runtimes", runtimes, flush=True)
spec = SG.column_scene(seed=cfg["seed"], n=cfg["n"], sweeps=cfg["sweeps"])
stream = torch.cuda.Stream()
alloc, free = T.torch_allocator()
before = torch.cuda.memory_allocated()
n = len(spec["x"])
bounds = np.array([list(spec["grid_lo"]) + list(spec["grid_hi"])], dtype=np.float64)
sc = T.Scene(n_envs=1, dt=spec["dt"], gravity=spec["gravity"], max_sweeps=spec["max_sweeps"], warm_start="prev",
             material=spec["material"], cap_particles=n, cap_contacts=16 * n, env_bounds=bounds,
             r_ref=spec["r_ref"], stream=stream.cuda_stream, alloc_fn=alloc, free_fn=free)
held = torch.cuda.memory_allocated() - before
sc.add_particles(0, spec["x"], spec["r"])
sc.set_kinematic_bodies(0, [dict(b, id=i) for i, b in enumerate(spec["bodies"])])
sc.step(cfg["steps"])
p = sc.get_particles(0)
keys, lam = sc.get_contacts(0)
sc.close()
released = before - torch.cuda.memory_allocated()
rng = np.random.default_rng(cfg["seed"])
W = torch.tensor(rng.normal(0, 0.2, T.MLP_PARAMS).astype(np.float32), device="cuda")
F = torch.tensor(rng.normal(0, 1.0, (cfg["batch"], 12)).astype(np.float32), device="cuda")
out = torch.zeros((cfg["batch"], 3), dtype=torch.float32, device="cuda")
torch.cuda.synchronize()
T.mlp_forward(W.data_ptr(), F.data_ptr(), cfg["batch"], out.data_ptr(), bf16=True, stream=stream.cuda_stream)
stream.synchronize()
np.savez(sys.argv[2], x=p["x"], v=p["v"], w=p["w"], keys=keys, lam=lam, mlp=out.cpu().numpy(),
         held=held, released=released, n_runtimes=len(runtimes), torch_runtime=int(all("torch" in r for r in runtimes)))
print("ok", flush=True)
"""


def test_scene_and_network_on_pytorch_memory_and_stream(tmp_path):
    cfg = dict(seed=7, n=800, sweeps=30, steps=4, batch=777)
    out = tmp_path / "child.npz"
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, str(out), json.dumps(cfg)], capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    got = np.load(out)
    assert int(got["n_runtimes"]) == 1 and int(got["torch_runtime"]) == 1, r.stdout
    assert int(got["held"]) > 0                  # the scene's buffers came from PyTorch's allocator
    assert int(got["released"]) == 0             # and went back to it at destroy_scene

    # the same work here, on the library's own runtime
    spec = SG.column_scene(seed=cfg["seed"], n=cfg["n"], sweeps=cfg["sweeps"])
    n = len(spec["x"])
    bounds = np.array([list(spec["grid_lo"]) + list(spec["grid_hi"])], dtype=np.float64)
    sc = T.Scene(n_envs=1, dt=spec["dt"], gravity=spec["gravity"], max_sweeps=spec["max_sweeps"], warm_start="prev",
                 material=spec["material"], cap_particles=n, cap_contacts=16 * n, env_bounds=bounds,
                 r_ref=spec["r_ref"])
    sc.add_particles(0, spec["x"], spec["r"])
    sc.set_kinematic_bodies(0, [dict(b, id=i) for i, b in enumerate(spec["bodies"])])
    sc.step(cfg["steps"])
    p = sc.get_particles(0)
    keys, lam = sc.get_contacts(0)
    sc.close()
    assert np.array_equal(got["keys"], keys) and np.array_equal(got["lam"], lam)
    for k in ("x", "v", "w"):
        assert np.array_equal(got[k], p[k]), k

    rng = np.random.default_rng(cfg["seed"])
    W = D.DeviceArray.from_host(rng.normal(0, 0.2, T.MLP_PARAMS).astype(np.float32))
    F = D.DeviceArray.from_host(rng.normal(0, 1.0, (cfg["batch"], 12)).astype(np.float32))
    o = D.DeviceArray((cfg["batch"], 3), np.float32)
    T.mlp_forward(W.ptr, F.ptr, cfg["batch"], o.ptr, bf16=True)
    assert np.array_equal(got["mlp"], o.get())
