"""Learned kernel-variant selector (an extension beyond the paper).

For an operation (SDDMM, SpMM, or the fused pass) on a plan, a small
multilayer perceptron maps the block's sparsity features (``plan_features``:
a log2 row-length histogram weighted by entries, the longest row, sizes,
average degree, kz and the operand type) to the predicted slowdown
log2(t_v / t_best) of every candidate variant v; the selector runs the least
predicted among the variants valid for (op, kz, dtype).

Training labels are the exhaustive autotuner's timings, and the network is
trained on the GPU by the library's own kernels (``mlp_linear_fwd``,
``mlp_linear_bwd``, ``mlp_mse``, ``mlp_adam``).  The autotuner stays the
fallback: for a block whose features fall outside the range seen in training
the selector times the candidates instead of predicting.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import spc3d as spc
from . import synth
from . import tune

NFEAT = spc.NFEAT
TARGET_CAP = 3.0  # slowdowns beyond 8x are all "bad"; capping keeps them from dominating the loss
# The library default (variant -1) is kept unless another candidate is
# predicted faster by more than this (log2 of 1.03: about the spread of
# repeated timings of one call).
KEEP_DEFAULT_MARGIN = math.log2(1.03)
# Margins tried per operation on the training blocks after the fit (log2 of
# the predicted speed-up a candidate must show over the default); inf keeps
# the default always, for an operation whose default the network cannot beat.
MARGIN_GRID = (0.0, math.log2(1.02), math.log2(1.03), math.log2(1.05), math.log2(1.08),
               math.log2(1.12), math.inf)


def candidates(op: str) -> list:
    """The network's outputs for op: the library default shape (-1) first,
    then every explicit variant the autotuner times."""
    return [-1] + tune.candidates(op)


class MLP:
    """Dense ReLU network with FP32 parameters on the device.

    sizes = [fin, h1, ..., fout]; ReLU after every layer but the last.
    Weights are initialised U(-sqrt(6/fin), sqrt(6/fin)) from the seeded
    counter generator, biases at zero.
    """

    def __init__(self, sizes, seed: int, device):
        self.sizes = list(sizes)
        self.device = torch.device(device)
        self.W, self.b = [], []
        for li, (fin, fout) in enumerate(zip(sizes[:-1], sizes[1:])):
            u = synth.uniform_f32(seed, fout * fin, ctr0=li << 32).astype(np.float32)
            w = torch.from_numpy(u.reshape(fout, fin) * np.float32(math.sqrt(6.0 / fin)))
            self.W.append(w.to(self.device))
            self.b.append(torch.zeros(fout, dtype=torch.float32, device=self.device))
        self.params = [p for pair in zip(self.W, self.b) for p in pair]
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.t = 0
        self._buf = None

    @property
    def nlayers(self) -> int:
        return len(self.W)

    def forward(self, X: torch.Tensor) -> list:
        """Activations [X, h1, ..., out] (each a new device tensor)."""
        acts = [X.contiguous()]
        for i in range(self.nlayers):
            acts.append(spc.mlp_linear_fwd(acts[-1], self.W[i], self.b[i],
                                           relu=i + 1 < self.nlayers))
        return acts

    def predict(self, X: torch.Tensor) -> torch.Tensor:
        return self.forward(X)[-1]

    def loss_and_grads(self, X, T, M):
        """Masked MSE of the output against T, and [(dW, db), ...] per layer."""
        acts = self.forward(X)
        loss, d = spc.mlp_mse(acts[-1], T, M)
        grads = [None] * self.nlayers
        n = X.shape[0]
        need = max(spc.mlp_linear_bwd_buffer_size(n, fi, fo)
                   for fi, fo in zip(self.sizes[:-1], self.sizes[1:]))
        if self._buf is None or self._buf.numel() < need:
            self._buf = torch.empty(need, dtype=torch.uint8, device=self.device)
        for i in range(self.nlayers - 1, -1, -1):
            dX, dW, db = spc.mlp_linear_bwd(acts[i], self.W[i], acts[i + 1], d,
                                            relu=i + 1 < self.nlayers, need_dx=i > 0,
                                            buf=self._buf)
            grads[i] = (dW, db)
            d = dX
        return loss, grads

    def step(self, grads, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        flat = [g for pair in grads for g in pair]
        for p, g, m, v in zip(self.params, flat, self.m, self.v):
            spc.mlp_adam(p, g, m, v, lr, beta1, beta2, eps, self.t)

    def fit(self, X, T, M, steps: int, lr: float, lr_final: float | None = None,
            log_every: int = 0, log=None) -> list:
        """Full-batch Adam; the learning rate decays geometrically to lr_final.
        Returns the loss every log_every steps (read back from the device)."""
        hist = []
        lr_final = lr if lr_final is None else lr_final
        for s in range(steps):
            a = lr * (lr_final / lr) ** (s / max(steps - 1, 1))
            loss, grads = self.loss_and_grads(X, T, M)
            self.step(grads, a)
            if log_every and (s % log_every == 0 or s == steps - 1):
                hist.append((s, float(loss.item())))
                if log:
                    log(f"  step {s:5d} loss {hist[-1][1]:.5f}")
        return hist

    def state(self) -> dict:
        return dict(sizes=self.sizes, W=[w.cpu().numpy().tolist() for w in self.W],
                    b=[b.cpu().numpy().tolist() for b in self.b])

    @classmethod
    def from_state(cls, st: dict, device) -> "MLP":
        m = cls(st["sizes"], 0, device)
        for i in range(m.nlayers):
            m.W[i].copy_(torch.tensor(st["W"][i], dtype=torch.float32))
            m.b[i].copy_(torch.tensor(st["b"][i], dtype=torch.float32))
        return m


def valid_mask(op: str, kz: int, dtype: int, cands=None) -> np.ndarray:
    """1.0 for the candidates of op that can run with (kz, dtype), else 0.0."""
    cands = candidates(op) if cands is None else cands
    return np.array([1.0 if tune.valid(op, kz, dtype, v) else 0.0 for v in cands],
                    dtype=np.float32)


def targets(timings: dict, op: str, cands=None):
    """Training row of one autotune result: (T, M) over the candidates of op,
    T = min(log2(t_v / t_best), TARGET_CAP) where timed, M = 1 there."""
    cands = candidates(op) if cands is None else cands
    best = min(t for v, t in timings.items() if v in cands)
    T = np.zeros(len(cands), np.float32)
    M = np.zeros(len(cands), np.float32)
    for k, v in enumerate(cands):
        if v in timings:
            T[k] = min(math.log2(timings[v] / best), TARGET_CAP)
            M[k] = 1.0
    return T, M


class Selector:
    """One MLP per operation, plus the feature range seen in training."""

    def __init__(self, hidden=(64, 64), seed: int = 7, device="cuda",
                 margin: float = KEEP_DEFAULT_MARGIN):
        self.hidden = tuple(hidden)
        self.margin = margin
        self.margins = {}   # op -> keep-default margin chosen on the training blocks
        self.seed = seed
        self.device = torch.device(device)
        self.models = {}
        self.cands = {}   # op -> candidate variants, one network output each
        self.lo = {}
        self.hi = {}
        self._masks = {}

    def fit(self, op: str, X: np.ndarray, T: np.ndarray, M: np.ndarray, steps: int = 3000,
            lr: float = 3e-3, lr_final: float = 3e-4, log_every: int = 0, log=None) -> list:
        X = np.asarray(X, np.float32)
        self.cands[op] = candidates(op)
        ncand = len(self.cands[op])
        assert X.shape[1] == NFEAT and T.shape[1] == ncand and M.shape == T.shape
        mlp = MLP([NFEAT, *self.hidden, ncand], self.seed + tune.OPCODE[op], self.device)
        dev = self.device
        hist = mlp.fit(torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev).contiguous(),
                       torch.from_numpy(M).to(dev).contiguous(), steps, lr, lr_final,
                       log_every, log)
        self.models[op] = mlp
        self.lo[op] = X.min(axis=0)
        self.hi[op] = X.max(axis=0)
        return hist

    def _mask(self, op, kz, dtype):
        key = (op, kz, dtype)
        if key not in self._masks:
            self._masks[key] = torch.from_numpy(valid_mask(op, kz, dtype, self.cands[op])).to(
                self.device)
        return self._masks[key]

    def margin_for(self, op: str) -> float:
        return self.margins.get(op, self.margin)

    def predict_indices(self, op: str, X: torch.Tensor, masks: torch.Tensor,
                        margin: float | None = None) -> torch.Tensor:
        """Per row of X, the index into self.cands[op] of the least
        predicted slowdown among the allowed ones (device int32, -1 if none);
        the default shape is kept unless beaten by more than the operation's
        margin (an infinite margin keeps it always)."""
        m = self.margin_for(op) if margin is None else margin
        pref = self.cands[op].index(-1) if -1 in self.cands[op] else -1
        if math.isinf(m) and pref >= 0:
            return torch.full((X.shape[0],), pref, dtype=torch.int32, device=X.device)
        P = self.models[op].predict(X)
        return spc.mlp_masked_argmin(P, masks.contiguous(), pref=pref, margin=m)

    def fit_margin(self, op: str, recs: list, grid=MARGIN_GRID) -> float:
        """Chooses the operation's keep-default margin on training records: the
        one of the grid with the least geometric-mean regret against the
        autotuner (ties go to the larger margin)."""
        rs = [r for r in recs if r["op"] == op]
        X = torch.from_numpy(np.stack([r["features"] for r in rs]).astype(np.float32)).to(
            self.device)
        masks = torch.from_numpy(np.stack([valid_mask(op, r["kz"], r["dtype"], self.cands[op])
                                           for r in rs])).to(self.device)
        best, best_reg = None, None
        for m in grid:
            idx = self.predict_indices(op, X, masks, margin=m).cpu().numpy()
            logs = []
            for r, k in zip(rs, idx):
                t = r["timings"]
                v = self.cands[op][k] if k >= 0 else -1
                logs.append(math.log(t.get(v, t[-1]) / min(t.values())))
            reg = float(np.mean(logs))
            if best_reg is None or reg <= best_reg:
                best, best_reg = m, reg
        self.margins[op] = best
        return best

    def in_range(self, op: str, f: np.ndarray, margin: float = 0.0) -> bool:
        """True when every feature lies within the training range (+- margin).
        No margin by default: just past the largest training blocks (the
        3D-share block's 430K rows against at most 2^18 in training, 0.045
        beyond the range in the scaled log2 of the row count) a network
        trained on the selector workload picked a shape 15% slower than the
        default, so such blocks go to the autotuner."""
        return bool(np.all(f >= self.lo[op] - margin) and np.all(f <= self.hi[op] + margin))

    def choose(self, plan, op: str, kz: int, dtype: int, vals=None, A=None, B=None):
        """(variant, source): source "mlp", or "autotune" when the model is
        absent or the block is outside its training range (A and B are then
        needed to time the candidates)."""
        feats = spc.plan_features(plan, kz, dtype)
        if op in self.models and self.in_range(op, feats.cpu().numpy()):
            idx = int(self.predict_indices(op, feats.view(1, NFEAT),
                                           self._mask(op, kz, dtype).view(1, -1)).item())
            if idx >= 0:
                return self.cands[op][idx], "mlp"
        if A is None or B is None:
            raise ValueError("the autotune fallback needs A and B")
        return tune.best_variant(tune.autotune(plan, op, vals, A, B, kz)), "autotune"

    def state(self) -> dict:
        return dict(hidden=list(self.hidden), seed=self.seed,
                    models={op: m.state() for op, m in self.models.items()},
                    cands={op: list(c) for op, c in self.cands.items()},
                    lo={op: v.tolist() for op, v in self.lo.items()},
                    hi={op: v.tolist() for op, v in self.hi.items()},
                    margins={op: (None if math.isinf(m) else m)
                             for op, m in self.margins.items()})

    @classmethod
    def from_state(cls, st: dict, device="cuda") -> "Selector":
        s = cls(st["hidden"], st["seed"], device)
        for op, ms in st["models"].items():
            s.models[op] = MLP.from_state(ms, device)
            s.cands[op] = list(st["cands"][op])
            s.lo[op] = np.array(st["lo"][op], np.float32)
            s.hi[op] = np.array(st["hi"][op], np.float32)
        for op, m in st.get("margins", {}).items():
            s.margins[op] = math.inf if m is None else float(m)
        return s


# ------------------------------------------------------------ data and judge

def collect(blocks, ks=(16, 32, 64, 128), dtypes=(spc.F32, spc.BF16), ops=tune.OPS,
            reps: int = 5, seed: int = synth.SELECTOR_SEED, device="cuda", log=None) -> list:
    """Autotune every (block, kz, dtype, op) instance.

    blocks: iterable of synth.selector_block dicts.  Returns records
    dict(block, kind, n, nnz, kz, dtype, op, features [NFEAT], timings
    {variant: ms}) where variant -1 is the library's default shape.
    """
    recs = []
    dev = torch.device(device)
    for blk in blocks:
        rows = torch.from_numpy(blk["rows"]).to(dev)
        cols = torch.from_numpy(blk["cols"]).to(dev)
        n = blk["n"]
        plan = spc.plan_create_coo(rows, cols, (0, n), (0, n))
        kmax = max(ks)
        vals = torch.from_numpy(synth.uniform_f32(seed + 7, plan.nnz, ctr0=blk["i"] << 36)).to(dev)
        Af = torch.from_numpy(synth.uniform_f32(seed + 101, plan.R * kmax, ctr0=blk["i"] << 36))
        Bf = torch.from_numpy(synth.uniform_f32(seed + 202, plan.C * kmax, ctr0=blk["i"] << 36))
        Af = Af.view(plan.R, kmax).to(dev)
        Bf = Bf.view(plan.C, kmax).to(dev)
        for kz in ks:
            for dt in dtypes:
                tdt = torch.float32 if dt == spc.F32 else torch.bfloat16
                A = Af[:, :kz].contiguous().to(tdt)
                B = Bf[:, :kz].contiguous().to(tdt)
                feats = spc.plan_features(plan, kz, dt).cpu().numpy()
                for op in ops:
                    t = tune.autotune(plan, op, vals, A, B, kz, reps=reps)
                    recs.append(dict(block=blk["i"], kind=blk["kind"], n=n, nnz=plan.nnz, kz=kz,
                                     dtype=dt, op=op, features=feats, timings=t))
        if log:
            log(f"block {blk['i']:4d} {blk['kind']:7s} n={n:7d} nnz={plan.nnz:9d} done "
                f"({len(recs)} records)")
        del plan
    return recs


def dataset(recs: list, op: str, cands=None):
    """(X, T, M) arrays of the records of op over its candidates (the
    network's outputs, candidates(op), unless given)."""
    rs = [r for r in recs if r["op"] == op]
    X = np.stack([r["features"] for r in rs]).astype(np.float32)
    TM = [targets(r["timings"], op, cands) for r in rs]
    return X, np.stack([t for t, _ in TM]), np.stack([m for _, m in TM])


def best_fixed(recs: list, op: str) -> int:
    """The single candidate with the least geometric-mean slowdown over the
    records of op, among those that run on every instance (if none does, an instance where a
    candidate cannot run counts the default's slowdown)."""
    recs = [r for r in recs if r["op"] == op]
    best, best_score = -1, None
    everywhere = [v for v in tune.candidates(op) if all(v in r["timings"] for r in recs)]
    for v in everywhere or tune.candidates(op):
        s = 0.0
        for r in recs:
            t = r["timings"]
            tb = min(t.values())
            s += math.log(t.get(v, t[-1]) / tb)
        if best_score is None or s < best_score:
            best, best_score = v, s
    return best


def judge(sel: Selector, recs: list, op: str, fixed: int | None = None) -> dict:
    """Regret of the selector on recs against the exhaustive autotuner, and its
    gain over the library default and over one fixed variant."""
    rs = [r for r in recs if r["op"] == op]
    X = torch.from_numpy(np.stack([r["features"] for r in rs]).astype(np.float32)).to(sel.device)
    cands = sel.cands[op]
    masks = torch.from_numpy(np.stack([valid_mask(op, r["kz"], r["dtype"], cands)
                                       for r in rs])).to(sel.device)
    idx = sel.predict_indices(op, X, masks).cpu().numpy()
    reg, g_def, g_fix, r_def, r_fix, hits = [], [], [], [], [], 0
    for r, k in zip(rs, idx):
        t = r["timings"]
        tb = min(t.values())
        v = cands[k] if k >= 0 else -1
        ts = t.get(v, t[-1])
        reg.append(ts / tb - 1.0)
        g_def.append(t[-1] / ts)
        r_def.append(t[-1] / tb - 1.0)
        if fixed is not None:
            tf = t.get(fixed, t[-1])
            g_fix.append(tf / ts)
            r_fix.append(tf / tb - 1.0)
        hits += ts == tb

    def gm(x):
        return float(math.exp(np.mean(np.log(x)))) if len(x) else float("nan")

    out = dict(op=op, n=len(rs),
               regret_geomean=gm(np.array(reg) + 1.0) - 1.0,
               regret_p90=float(np.percentile(reg, 90)),
               regret_max=float(np.max(reg)),
               top1=hits / len(rs),
               default_regret_geomean=gm(np.array(r_def) + 1.0) - 1.0,
               default_regret_p90=float(np.percentile(r_def, 90)),
               gain_vs_default_geomean=gm(g_def))
    if fixed is not None:
        out.update(fixed_variant=fixed,
                   fixed_regret_geomean=gm(np.array(r_fix) + 1.0) - 1.0,
                   gain_vs_fixed_geomean=gm(g_fix))
    return out


def save_weights(state: dict, path: str, note: str = ""):
    """Write a Selector.state() compactly: FP32 arrays as base64 little-endian."""
    import base64
    import json

    def enc(a):
        a = np.asarray(a, dtype="<f4")
        return dict(shape=list(a.shape), b64=base64.b64encode(a.tobytes()).decode())

    out = dict(note=note, hidden=state["hidden"], seed=state["seed"], models={}, lo={}, hi={},
               cands=state["cands"], margins=state.get("margins", {}))
    for op, m in state["models"].items():
        out["models"][op] = dict(sizes=m["sizes"], W=[enc(w) for w in m["W"]],
                                 b=[enc(b) for b in m["b"]])
        out["lo"][op] = enc(state["lo"][op])
        out["hi"][op] = enc(state["hi"][op])
    with open(path, "w") as f:
        json.dump(out, f)


def load_weights(path: str) -> dict:
    """Inverse of save_weights: a state dict for Selector.from_state."""
    import base64
    import json

    def dec(d):
        return np.frombuffer(base64.b64decode(d["b64"]), dtype="<f4").reshape(d["shape"])

    with open(path) as f:
        w = json.load(f)
    st = dict(hidden=w["hidden"], seed=w["seed"], models={}, lo={}, hi={},
              cands=w.get("cands") or {op: _legacy_candidates(op) for op in w["models"]},
              margins=w.get("margins", {}))
    for op, m in w["models"].items():
        st["models"][op] = dict(sizes=m["sizes"], W=[dec(x).tolist() for x in m["W"]],
                                b=[dec(x).tolist() for x in m["b"]])
        st["lo"][op] = dec(w["lo"][op]).tolist()
        st["hi"][op] = dec(w["hi"][op]).tolist()
    return st


def _legacy_candidates(op: str) -> list:
    """Candidates of networks saved before the windowed SpMM family existed."""
    return [v for v in tune.GROUP_VARIANTS if op != "sddmm" or not (v >> 8) & 1]


def save_records(recs: list, path: str):
    import json
    rows = [dict(r, features=[float(x) for x in r["features"]],
                 timings={str(k): v for k, v in r["timings"].items()}) for r in recs]
    with open(path, "w") as f:
        json.dump(rows, f)


def load_records(path: str) -> list:
    import json
    with open(path) as f:
        rows = json.load(f)
    return [dict(r, features=np.array(r["features"], np.float32),
                 timings={int(k): v for k, v in r["timings"].items()}) for r in rows]


def save_records_npz(recs: list, path: str):
    """Records as compact arrays (one row per record, one timing column per
    variant of candidates("spmm"), NaN where a variant was not timed)."""
    cols = candidates("spmm")
    col = {v: i for i, v in enumerate(cols)}
    T = np.full((len(recs), len(cols)), np.nan, np.float32)
    for i, r in enumerate(recs):
        for v, t in r["timings"].items():
            T[i, col[v]] = t
    np.savez_compressed(path, variants=np.array(cols, np.int32), timings=T,
                        features=np.stack([r["features"] for r in recs]).astype(np.float32),
                        block=np.array([r["block"] for r in recs], np.int32),
                        kz=np.array([r["kz"] for r in recs], np.int32),
                        dtype=np.array([r["dtype"] for r in recs], np.int32),
                        op=np.array([r["op"] for r in recs]),
                        nnz=np.array([r["nnz"] for r in recs], np.int64),
                        kind=np.array([r["kind"] for r in recs]), n=np.array([r["n"] for r in recs]))


def load_records_npz(path: str) -> list:
    z = np.load(path, allow_pickle=False)
    cols = [int(v) for v in z["variants"]]
    out = []
    for i in range(z["timings"].shape[0]):
        row = z["timings"][i]
        out.append(dict(block=int(z["block"][i]), kind=str(z["kind"][i]), n=int(z["n"][i]),
                        nnz=int(z["nnz"][i]), kz=int(z["kz"][i]), dtype=int(z["dtype"][i]),
                        op=str(z["op"][i]), features=z["features"][i],
                        timings={v: float(row[k]) for k, v in enumerate(cols)
                                 if not np.isnan(row[k])}))
    return out


def main(argv=None):
    """Collect autotuner timings on the selector workload, train one MLP per
    operation on the training blocks, and judge it on the held-out blocks."""
    import argparse
    import json
    import sys
    import time

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--blocks", type=int, default=512)
    ap.add_argument("--train", type=int, default=384)
    ap.add_argument("--lg-hi", type=float, default=18.0, help="log2 of the largest block side")
    ap.add_argument("--deg-hi", type=float, default=64.0)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--time-limit", type=float, default=0.0,
                    help="stop timing new blocks after this many seconds (0: no limit)")
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--hidden", type=int, nargs="+", default=[64, 64])
    ap.add_argument("--data", help="load autotuner records from this JSON instead of timing")
    ap.add_argument("--save-data", help="write the autotuner records to this JSON")
    ap.add_argument("--out", help="write the report and the trained networks to this JSON")
    ap.add_argument("--weights", help="write the trained networks (compact) to this JSON")
    ap.add_argument("--save-heldout", help="write the held-out blocks' records (compact .npz)")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    t0 = time.time()
    if args.data:
        recs = load_records(args.data)
    else:
        torch.cuda.init()
        from concurrent.futures import ThreadPoolExecutor

        def blocks():
            # the next block is generated on the host while the current one is timed
            with ThreadPoolExecutor(1) as ex:
                gen = lambda i: synth.selector_block(i, lg_hi=args.lg_hi, deg_hi=args.deg_hi)
                fut = ex.submit(gen, 0)
                for i in range(args.blocks):
                    blk = fut.result()
                    if i + 1 < args.blocks:
                        fut = ex.submit(gen, i + 1)
                    if args.time_limit and time.time() - t0 > args.time_limit:
                        log(f"time limit: stopping after {i} blocks")
                        return
                    yield blk
        recs = collect(blocks(), log=log, reps=args.reps)
        if args.save_data:
            save_records(recs, args.save_data)
    log(f"{len(recs)} records ({time.time() - t0:.0f} s)")
    train, held = synth.selector_split(args.blocks, args.train)
    timed = {r["block"] for r in recs}
    train, held = set(train) & timed, set(held) & timed
    rtrain = [r for r in recs if r["block"] in train]
    rheld = [r for r in recs if r["block"] in held]
    if args.save_heldout:
        save_records_npz(rheld, args.save_heldout)
    sel = Selector(args.hidden)
    report = dict(blocks=len(timed), train_blocks=len(train), held_out_blocks=len(held),
                  steps=args.steps, hidden=args.hidden, reps=args.reps, ops={})
    for op in tune.OPS:
        X, T, M = dataset(rtrain, op)
        t1 = time.time()
        hist = sel.fit(op, X, T, M, steps=args.steps, log_every=max(args.steps // 6, 1), log=log)
        torch.cuda.synchronize()
        fit_s = time.time() - t1
        marg = sel.fit_margin(op, rtrain)
        log(f"{op:10s} keep-default margin chosen on the training blocks: "
            f"{'always the default' if math.isinf(marg) else f'{2 ** marg:.2f}x'}")
        fixed = best_fixed(rtrain, op)
        report["ops"][op] = dict(train=judge(sel, rtrain, op, fixed),
                                 held_out=judge(sel, rheld, op, fixed),
                                 loss=hist, fit_seconds=fit_s,
                                 margin=None if math.isinf(marg) else marg)
        h = report["ops"][op]["held_out"]
        log(f"{op:10s} held-out n={h['n']}: regret geomean {h['regret_geomean']:.4f} "
            f"p90 {h['regret_p90']:.4f} top1 {h['top1']:.3f} | default regret "
            f"{h['default_regret_geomean']:.4f} | gain vs default {h['gain_vs_default_geomean']:.4f}"
            f" vs fixed {h['gain_vs_fixed_geomean']:.4f} | fit {fit_s:.1f} s")
    if args.out:
        with open(args.out, "w") as f:
            json.dump(dict(report=report, selector=sel.state()), f)
    if args.weights:
        save_weights(sel.state(), args.weights,
                     note=f"trained on {len(train)} blocks of the selector workload "
                          f"({args.steps} Adam steps, hidden {args.hidden})")
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
