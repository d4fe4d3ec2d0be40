"""Learned warm start: dataset, GPU training, weights.

The network (12 inputs, two 64-wide SiLU layers, 3 outputs) predicts the
converged impulses of a contact, scaled by m_eff g dt and expressed in the
contact frame, from features of the contact and of its previous-step impulse
(the inputs are listed with `get_learn_samples` in the C header).  Its outputs
are corrections added to the previous-step impulse (the residual form the
library applies), so the training targets are converged minus previous.  It is
trained on contacts that the plain solver produces on the small loose-column
workload (1,000 spheres, r 0.05 m, mu 0.6, c 1 kPa), solved to a tight
residual so that the impulses are the converged ones.

Training runs on the GPU through the library's own forward/backward and Adam
kernels (`mlp_loss_grad`, `mlp_adam_step`) on device buffers of the HIP
runtime the library links.  The loss is 0.5 mean ||y - label||^2 over a
minibatch.
"""
import math

import numpy as np

from . import scenegen as SG
from . import terrain as T
from .devmem import DeviceArray

N_IN, N_HID, N_OUT = 12, 64, 3
LAYOUT = (("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,)), ("in_scale", (N_IN,)))


def flatten(w):
    """Dict of arrays -> the flat FP32 parameter vector the library takes."""
    return np.concatenate([np.asarray(w[k], dtype=np.float32).ravel() for k, _ in LAYOUT])


def unflatten(flat):
    out, o = {}, 0
    for k, shp in LAYOUT:
        n = int(np.prod(shp))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def init_weights(seed=0, in_scale=None):
    """Glorot-uniform weights, zero biases, and the input normalisation."""
    rng = np.random.default_rng(seed)

    def glorot(fo, fi):
        a = math.sqrt(6.0 / (fi + fo))
        return rng.uniform(-a, a, (fo, fi))

    w = dict(W1=glorot(N_HID, N_IN), b1=np.zeros(N_HID), W2=glorot(N_HID, N_HID), b2=np.zeros(N_HID),
             W3=glorot(N_OUT, N_HID) * 0.1, b3=np.zeros(N_OUT),
             in_scale=np.ones(N_IN) if in_scale is None else np.asarray(in_scale, dtype=np.float64))
    return w


def input_scale(feat):
    """Per-feature normalisation: 1 / RMS over the dataset (1 for constant features)."""
    rms = np.sqrt(np.mean(np.asarray(feat, dtype=np.float64) ** 2, axis=0))
    return np.where(rms > 1e-12, 1.0 / np.maximum(rms, 1e-12), 1.0)


def column_batch(n_envs, seed, n=1000, sweeps=100, tol=0.0, warm="prev"):
    """Loose columns of the small workload, one per env (seeds seed .. seed + n_envs - 1)."""
    specs = [SG.column_scene(seed=seed + e, n=n, sweeps=sweeps) for e in range(n_envs)]
    return [dict(s, tol=tol, warm_start=warm) for s in specs]


def gen_dataset(n_envs=16, steps=120, skip=8, seed=100, tol=1e-5, max_sweeps=4000, cap=2_000_000, log=None):
    """Features and converged impulses (`get_learn_samples`) from column
    trajectories stepped on the GPU with the previous-step warm start and a
    tight residual tolerance.  The first `skip` steps (free fall, few contacts)
    and env-steps stopped by the sweep cap are not recorded; when the
    trajectories hold more than `cap` samples, a seeded uniform subset is
    kept."""
    specs = column_batch(n_envs, seed, sweeps=max_sweeps, tol=tol)
    sc = T.scene_from_specs(specs)
    sc.set_learn_capture(True)
    feats, labels, total = [], [], 0
    for k in range(steps):
        st = sc.step(1)
        if k < skip:
            continue
        for e in range(n_envs):
            if st[e]["sweeps"] >= max_sweeps:
                continue  # stopped by the cap, not by the tolerance
            f, lab = sc.get_learn_samples(e)
            feats.append(f)
            labels.append(lab)
            total += len(f)
        if log and k % 10 == 0:
            log(f"dataset step {k}: {total} samples, mean sweeps {np.mean([s['sweeps'] for s in st]):.0f}")
    sc.close()
    feat = np.concatenate(feats)
    label = np.concatenate(labels)
    ok = np.all(np.isfinite(feat), axis=1) & np.all(np.isfinite(label), axis=1)
    feat, label = feat[ok], label[ok]
    if len(feat) > cap:
        keep = np.sort(np.random.default_rng(seed).choice(len(feat), cap, replace=False))
        feat, label = feat[keep], label[keep]
    return feat, label


def gen_bed_dataset(n_envs=32, steps=60, skip=20, seed=7000, tol=1e-5, max_sweeps=4000, cap=2_000_000, log=None):
    """Features and converged impulses from beds of the batched workload's
    distribution (`scenegen.batch_specs` with seeds seed .. seed + n_envs - 1,
    disjoint from the evaluation beds), their tools moving, stepped on the GPU
    with the previous-step start and a tight residual tolerance; the first
    `skip` steps (the pour) are not recorded, nor the env-steps that reached
    the sweep cap before the tolerance."""
    specs = SG.batch_specs(seed=seed, n_envs=n_envs, sweeps=max_sweeps)
    mat = specs[0]["material"]
    specs = [dict(s, material=mat, tol=tol, warm_start="prev") for s in specs]
    nmax = max(len(s["x"]) for s in specs)
    sc = T.scene_from_specs(specs, cap_particles=nmax, cap_contacts=8 * nmax)
    sc.set_learn_capture(True)
    feats, labels, total = [], [], 0
    for k in range(steps):
        st = sc.step(1)
        if k < skip:
            continue
        for e in range(n_envs):
            if st[e]["sweeps"] >= max_sweeps:
                continue  # stopped by the cap, not by the tolerance: its impulses are not converged
            f, lab = sc.get_learn_samples(e)
            feats.append(f)
            labels.append(lab)
            total += len(f)
        if log and k % 10 == 0:
            log(f"bed dataset step {k}: {total} samples, mean sweeps {np.mean([s['sweeps'] for s in st]):.0f}")
    sc.close()
    feat, label = np.concatenate(feats), np.concatenate(labels)
    ok = np.all(np.isfinite(feat), axis=1) & np.all(np.isfinite(label), axis=1)
    feat, label = feat[ok], label[ok]
    if len(feat) > cap:
        keep = np.sort(np.random.default_rng(seed).choice(len(feat), cap, replace=False))
        feat, label = feat[keep], label[keep]
    return feat, label


def gen_mixed_dataset(seed=100, cap=2_000_000, log=None):
    """Half the samples from column trajectories (the small workload), half
    from beds of the batched workload's distribution: the contacts the plain
    solver produces on the scenes the start is judged on."""
    fc, lc = gen_dataset(seed=seed, cap=cap // 2, log=log)
    fb, lb = gen_bed_dataset(seed=7000 + seed, cap=cap - len(fc), log=log)
    return np.concatenate([fc, fb]), np.concatenate([lc, lb])


def residual_targets(feat, label):
    """Training targets of the residual form: converged impulse minus the
    previous-step impulse (inputs 3-5), both in the contact frame / (m_eff g dt)."""
    return (np.asarray(label, dtype=np.float64) - np.asarray(feat, dtype=np.float64)[:, 3:6]).astype(np.float32)


class Trainer:
    """Adam on the GPU over a dataset resident in device memory.  Each epoch
    visits the samples in a fresh seeded order (shuffled on the host and
    uploaded, about 60 B per sample)."""

    def __init__(self, weights, feat, label, batch=4096, seed=0):
        self.feat_h = np.ascontiguousarray(feat, dtype=np.float32)
        self.label_h = np.ascontiguousarray(label, dtype=np.float32)
        n = T.MLP_TRAINABLE
        self.W = DeviceArray.from_host(flatten(weights))
        self.G, self.M, self.V = DeviceArray(n), DeviceArray(n), DeviceArray(n)
        self.M.zero()
        self.V.zero()
        self.L = DeviceArray(1)
        self.feat = DeviceArray(self.feat_h.shape)
        self.label = DeviceArray(self.label_h.shape)
        self.batch = batch
        self.ns = T.mlp_grad_scratch_floats(batch)
        self.S = DeviceArray(max(self.ns, 1))
        self.t = 0
        self.rng = np.random.default_rng(seed)
        # a fixed minibatch for the gradient check
        k = min(256, len(self.feat_h))
        self.check_f = DeviceArray.from_host(self.feat_h[:k])
        self.check_l = DeviceArray.from_host(self.label_h[:k])

    def loss_grad(self, fptr, lptr, B):
        """Loss and gradient of one minibatch (device pointers) into L / G."""
        T.mlp_loss_grad(self.W.ptr, fptr, lptr, B, self.G.ptr, self.L.ptr, self.S.ptr, self.ns)

    def epoch(self, lr):
        perm = self.rng.permutation(len(self.feat_h))
        self.feat.upload(self.feat_h[perm])
        self.label.upload(self.label_h[perm])
        losses = []
        for i in range(0, len(perm) - self.batch + 1, self.batch):
            self.loss_grad(self.feat.at(i), self.label.at(i), self.batch)
            losses.append(float(self.L.get()[0]))  # every minibatch: the targets are heavy-tailed
            self.t += 1
            T.mlp_adam_step(self.W.ptr, self.G.ptr, self.M.ptr, self.V.ptr, lr, self.t)
        return float(np.mean(losses)) if losses else float(self.L.get()[0])

    def fit(self, epochs=20, lr=2e-3, lr_end=2e-4, check=None, log=None):
        """Geometric learning-rate decay from lr to lr_end.  After every epoch
        `check(weights, feat, label, grad, loss)` gets a fixed minibatch and the
        GPU gradient on it (the caller's gradient check)."""
        hist = []
        for ep in range(epochs):
            a = lr * (lr_end / lr) ** (ep / max(epochs - 1, 1))
            loss = self.epoch(a)
            hist.append(loss)
            if check is not None:
                k = self.check_f.shape[0]
                self.loss_grad(self.check_f.ptr, self.check_l.ptr, k)
                check(self.weights(), self.check_f.get(), self.check_l.get(), self.G.get(), float(self.L.get()[0]))
            if log:
                log(f"epoch {ep}: loss {loss:.5f} lr {a:.2e}")
        return hist

    def weights(self):
        return self.W.get().copy()

    def mean_loss(self, feat, label):
        """Mean loss over a held-out set (FP32 forward kernel)."""
        f = DeviceArray.from_host(feat)
        out = DeviceArray((len(feat), 3))
        T.mlp_forward(self.W.ptr, f.ptr, len(feat), out.ptr, bf16=False)
        y = out.get().astype(np.float64)
        f.free()
        out.free()
        return float(0.5 * np.mean(np.sum((y - label) ** 2, axis=1)))


def sweeps_to_tol(specs, modes=("cold", "prev", "learned"), weights=None, settle=40, steps=20, tol=1e-4,
                  max_sweeps=3000, bf16=True, schedule=None, graphs=True):
    """For each warm start: mean PGS sweeps per step to reach R_k <= tol, and
    steps/s, over `steps` steps of a batch of envs.  Every mode starts from the
    same state: the envs are first stepped `settle` steps (previous-step start)
    and that state, with its contact cache, is restored before each mode."""
    import time
    sp = [dict(s, warm_start="prev", tol=tol, max_sweeps=max_sweeps) for s in specs]
    sc = T.scene_from_specs(sp)
    if schedule:
        sc.set_solver_config(**schedule)
    sc.set_step_graphs(graphs)
    if weights is not None:
        sc.set_mlp_weights(weights)
        sc.set_learned_precision(bf16)
    sc.step(settle, stats=False)
    state = sc.save_state()
    out = {}
    for mode in modes:
        sc.load_state(state)
        sc.set_warm_start(mode)
        sweeps, capped, fallback = [], 0, 0
        stats = []
        t0 = time.perf_counter()
        for _ in range(steps):
            st = sc.step(1)
            stats.append(st)
        wall = time.perf_counter() - t0
        for st in stats:
            sweeps.extend(x["sweeps"] for x in st)
            capped += sum(x["sweeps"] >= max_sweeps for x in st)
            fallback += sum(x["fallback_used"] for x in st)
        edges = [0, 10, 30, 100, 300, 1000, 3000, max_sweeps, max_sweeps + 1]
        hist, _ = np.histogram(sweeps, bins=edges)
        out[mode] = dict(mean_sweeps=float(np.mean(sweeps)), steps_per_s=steps / wall, capped=int(capped),
                         capped_frac=float(capped) / max(len(sweeps), 1), fallback=int(fallback),
                         env_steps=len(sweeps), steps=steps,
                         sweep_histogram={"edges": edges, "counts": [int(c) for c in hist]})
        if mode == "learned":
            out[mode]["learned_kept"] = len(sweeps) - int(fallback)
    sc.close()
    return out


def main():
    import argparse
    import os
    ap = argparse.ArgumentParser(description="generate the dataset and train the learned warm start on the GPU")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "weights", "warmstart_column.npy"))
    ap.add_argument("--envs", type=int, default=16)
    ap.add_argument("--steps", type=int, default=120)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--samples", type=int, default=2_000_000)
    args = ap.parse_args()
    log = lambda m: print(m, flush=True)  # noqa: E731
    feat, label = gen_dataset(n_envs=args.envs, steps=args.steps, cap=args.samples, log=log)
    log(f"dataset: {len(feat)} samples")
    w = init_weights(0, input_scale(feat))
    tr = Trainer(w, feat, residual_targets(feat, label))
    tr.fit(epochs=args.epochs, log=log)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.save(args.out, tr.weights())
    log(f"weights: {args.out}")


if __name__ == "__main__":
    main()
