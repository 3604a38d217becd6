"""Learned kernel selector: a small MLP cost model choosing, per (form, degree, mesh size),
between the tensor-representation kernel (in several launch shapes) and the quadrature
kernel -- the automatic choice between the two approaches that Sec. 4.4 leaves open.

* features: form rank, degree q, log2 |i| (element tensor entries), log2(|alpha| + 1),
  dimension, log2(cells), log2(cells |i|) (output entries);
* output: predicted log(t_c / t_default) of every candidate launch c of
  ``tune.CANDIDATES_FP64`` relative to the library default launch (candidate 0); the choice
  is the argmin (the default itself predicts ~0), so the network only has to learn where
  and by how much a launch beats the default;
* training data: the autotuner's sweep (``tune.sweep``), whose exhaustive minimum is also
  the judge: regret = t_chosen / t_best - 1;
* training runs on the GPU through the library's own MLP forward, backward, MSE and Adam
  kernels (``ffc_mlp_*`` in include/ffc_hip.h), with an L2 weight penalty (the sweeps give
  a few hundred noisy timings; without it the network fits the noise); ``ref_forward`` /
  ``ref_backward`` are the plain FP64 NumPy statements of the same network that the tests
  check those kernels against.

Both kernels a choice can route to are exact to their stated tolerances, so the selector
changes speed, never results.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import capi
from .tune import CANDIDATES_FP64

N_FEATURES = 7


def features(kind: str, dim: int, degree: int, cells: int, n_I: int, n_alpha: int) -> np.ndarray:
    lc = math.log2(max(cells, 1))
    return np.array([2.0, degree, math.log2(n_I), math.log2(n_alpha + 1), dim, lc, lc + math.log2(n_I)],
                    dtype=np.float64)


# ----------------------------------------------------------- reference statement ---

def split_params(p: np.ndarray, n_in: int, h: int, n_out: int):
    o = 0
    W1 = p[o:o + n_in * h].reshape(n_in, h); o += n_in * h
    b1 = p[o:o + h]; o += h
    W2 = p[o:o + h * h].reshape(h, h); o += h * h
    b2 = p[o:o + h]; o += h
    W3 = p[o:o + h * n_out].reshape(h, n_out); o += h * n_out
    b3 = p[o:o + n_out]; o += n_out
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def ref_forward(p, x, n_in, h, n_out):
    """FP64 statement of the network: (y, (h1, h2))."""
    W1, b1, W2, b2, W3, b3 = split_params(np.asarray(p, np.float64), n_in, h, n_out)
    x = np.asarray(x, np.float64)
    h1 = np.maximum(x @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h2 @ W3 + b3, (h1, h2)


def ref_backward(p, x, dy, n_in, h, n_out):
    """FP64 gradient of sum(dy * y) w.r.t. the flat parameters."""
    W1, b1, W2, b2, W3, b3 = split_params(np.asarray(p, np.float64), n_in, h, n_out)
    x = np.asarray(x, np.float64)
    dy = np.asarray(dy, np.float64)
    _, (h1, h2) = ref_forward(p, x, n_in, h, n_out)
    gW3, gb3 = h2.T @ dy, dy.sum(0)
    d2 = (dy @ W3.T) * (h2 > 0)
    gW2, gb2 = h1.T @ d2, d2.sum(0)
    d1 = (d2 @ W2.T) * (h1 > 0)
    gW1, gb1 = x.T @ d1, d1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def ref_mse(y, t, m):
    m = np.asarray(m, np.float64)
    c = max(m.sum(), 1.0)
    d = (np.asarray(y, np.float64) - t) * m
    return float((d * d).sum() / c), 2.0 * d / c


# ------------------------------------------------------------------ GPU network ---

class MLP:
    """The selector network on the GPU; every step runs in the library's kernels."""

    def __init__(self, n_in=N_FEATURES, n_hidden=64, n_out=len(CANDIDATES_FP64), seed=0):
        import torch

        self.n_in, self.h, self.n_out = n_in, n_hidden, n_out
        L = capi.lib()
        self.n_params = int(L.ffc_mlp_param_count(n_in, n_hidden, n_out))
        rng = np.random.default_rng(seed)
        p = []
        for fan_in, fan_out in ((n_in, n_hidden), (n_hidden, n_hidden), (n_hidden, n_out)):
            p.append(rng.normal(0.0, math.sqrt(2.0 / fan_in), size=fan_in * fan_out))
            p.append(np.zeros(fan_out))
        self.params = torch.tensor(np.concatenate(p), dtype=torch.float32, device="cuda")
        assert self.params.numel() == self.n_params
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step_count = 0
        self.stream = torch.cuda.current_stream()

    def _s(self):
        return self.stream.cuda_stream

    def forward(self, x):
        """x: float32 CUDA tensor [batch, n_in] -> (y [batch, n_out], activations)."""
        import torch

        b = x.shape[0]
        act = torch.empty((2 * b * self.h,), dtype=torch.float32, device="cuda")
        y = torch.empty((b, self.n_out), dtype=torch.float32, device="cuda")
        capi.check(capi.lib().ffc_mlp_forward(self.n_in, self.h, self.n_out, b, self.params.data_ptr(), x.data_ptr(),
                                              act.data_ptr(), y.data_ptr(), self._s()))
        return y, act

    def backward(self, x, act, dy):
        import torch

        b = x.shape[0]
        work = torch.empty((2 * b * self.h,), dtype=torch.float32, device="cuda")
        capi.check(capi.lib().ffc_mlp_backward(self.n_in, self.h, self.n_out, b, self.params.data_ptr(), x.data_ptr(),
                                               act.data_ptr(), dy.data_ptr(), self.grad.data_ptr(), work.data_ptr(),
                                               self._s()))
        return self.grad

    def mse(self, y, t, m):
        import torch

        dy = torch.empty_like(y)
        loss = torch.empty((1,), dtype=torch.float32, device="cuda")
        capi.check(capi.lib().ffc_mlp_mse(y.numel(), y.data_ptr(), t.data_ptr(), m.data_ptr(), dy.data_ptr(),
                                          loss.data_ptr(), self._s()))
        return loss, dy

    def adam(self, lr=3e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        self.step_count += 1
        capi.check(capi.lib().ffc_adam_step(self.n_params, self.params.data_ptr(), self.grad.data_ptr(),
                                            self.m.data_ptr(), self.v.data_ptr(), ctypes.c_float(lr),
                                            ctypes.c_float(beta1), ctypes.c_float(beta2), ctypes.c_float(eps),
                                            ctypes.c_float(weight_decay), self.step_count, self._s()))

    def fit(self, X, Y, M, epochs=3000, lr=3e-3, weight_decay=0.0):
        """Full-batch training on (X features, Y targets, M masks) -> final loss."""
        import torch

        x = torch.tensor(X, dtype=torch.float32, device="cuda").contiguous()
        t = torch.tensor(Y, dtype=torch.float32, device="cuda").contiguous()
        m = torch.tensor(M, dtype=torch.float32, device="cuda").contiguous()
        loss = None
        for _ in range(epochs):
            y, act = self.forward(x)
            loss, dy = self.mse(y, t, m)
            self.backward(x, act, dy)
            self.adam(lr, weight_decay=weight_decay)
        torch.cuda.synchronize()
        return float(loss.item())

    def predict(self, X):
        import torch

        x = torch.tensor(X, dtype=torch.float32, device="cuda").contiguous()
        y, _ = self.forward(x)
        torch.cuda.synchronize()
        return y.cpu().numpy().astype(np.float64)


# ----------------------------------------------------------------- the selector ---

def records_to_arrays(records):
    """Features, targets log(t_c / t_0) and masks (0 where a timing is missing)."""
    X = np.stack([features(r["kind"], r["dim"], r["degree"], r["cells"], r["n_I"], r["n_alpha"]) for r in records])
    ok = lambda t: t is not None and t > 0  # noqa: E731
    T = np.array([[math.log(t / r["ms"][0]) if ok(t) and ok(r["ms"][0]) else 0.0 for t in r["ms"]]
                  for r in records])
    M = np.array([[1.0 if ok(t) and ok(r["ms"][0]) else 0.0 for t in r["ms"]] for r in records])
    return X, T, M


# A candidate replaces the default launch only if it is predicted faster by more than this
# fraction: the network's predictions carry errors of a few percent, and switching on a
# predicted gain below them picks slower launches about as often as faster ones.  Chosen by
# cross-validation over the stored sweep (mean regret and summed time at margins 0 .. 0.15,
# per-size folds and leave-one-form-out folds, both best at 0.01 - 0.02).
DECISION_MARGIN = 0.02


class Selector:
    """Normalised features -> MLP -> the candidate with the lowest predicted time relative to
    the default launch, if that beats the default by more than the decision margin."""

    def __init__(self, n_hidden=64, seed=0, margin=DECISION_MARGIN):
        self.net = MLP(n_hidden=n_hidden, seed=seed)
        self.mu = np.zeros(N_FEATURES)
        self.sd = np.ones(N_FEATURES)
        self.tmu = 0.0
        self.margin = margin

    def fit(self, records, epochs=3000, lr=3e-3, weight_decay=1e-3):
        X, T, M = records_to_arrays(records)
        self.mu, self.sd = X.mean(0), X.std(0) + 1e-9
        self.tmu = float((T * M).sum() / M.sum())
        return self.net.fit((X - self.mu) / self.sd, T - self.tmu, M, epochs, lr, weight_decay)

    def predict_rel(self, records):
        """Predicted log(t_c / t_default) per record and candidate."""
        X, _, _ = records_to_arrays(records)
        return self.net.predict((X - self.mu) / self.sd) + self.tmu

    def decide(self, pred, allowed=None) -> int:
        """The pick for one row of predict_rel: the lowest predicted candidate (among
        `allowed`, default all) if it beats the default (candidate 0) by more than the margin,
        else the default."""
        idx = range(len(pred)) if allowed is None else allowed
        j = min(idx, key=lambda i: pred[i])
        return int(j) if pred[j] < pred[0] - math.log1p(self.margin) else 0

    def choose(self, records):
        return [self.decide(y) for y in self.predict_rel(records)]

    def export(self, path, candidates=CANDIDATES_FP64):
        """Write the trained selector as the text file that the library's automatic kernel
        choice (FFC_KERNEL_AUTO) reads at form creation: sizes, feature normalisation, the
        offset of the targets, the decision margin, the flat FP32 parameters and the candidate
        launches, one per
        line as "kernel tile_cells waves persistent tile_window geometry" with kernel 1 =
        tensor, 2 = quadrature and geometry 0 = default, 1 = pass, 2 = fused."""
        from . import capi

        params = self.net.params.detach().cpu().numpy().astype(np.float32)
        lines = ["ffc_selector 2", f"n_in {self.net.n_in} n_hidden {self.net.h} n_out {self.net.n_out}",
                 "mu " + " ".join(repr(float(v)) for v in self.mu),
                 "sd " + " ".join(repr(float(v)) for v in self.sd),
                 f"tmu {self.tmu!r}", f"margin {float(self.margin)!r}",
                 f"params {params.size} " + " ".join(repr(float(v)) for v in params),
                 f"candidates {len(candidates)}"]
        for c in candidates:
            lines.append(" ".join(str(v) for v in (
                capi.KERNELS[c["kernel"]], c.get("tile_cells", 0), c.get("waves", 0), c.get("persistent", 0),
                c.get("tile_window", 0), capi.GEOMETRY[c.get("geometry", "default")])))
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            f.write("\n".join(lines) + "\n")
        os.replace(tmp, path)

    @classmethod
    def load(cls, path):
        """A selector with the parameters of a file written by export()."""
        import torch

        tok = open(path).read().split()
        assert tok[0] == "ffc_selector" and tok[1] in ("1", "2"), "not a selector file"
        version = int(tok[1])
        n_in, h, n_out = int(tok[3]), int(tok[5]), int(tok[7])
        assert n_in == N_FEATURES and n_out == len(CANDIDATES_FP64)
        i = 8
        assert tok[i] == "mu"
        mu = np.array([float(x) for x in tok[i + 1:i + 1 + n_in]]); i += 1 + n_in
        assert tok[i] == "sd"
        sd = np.array([float(x) for x in tok[i + 1:i + 1 + n_in]]); i += 1 + n_in
        assert tok[i] == "tmu"
        tmu = float(tok[i + 1]); i += 2
        margin = 0.0  # version 1 files: plain argmin
        if version == 2:
            assert tok[i] == "margin"
            margin = float(tok[i + 1]); i += 2
        assert tok[i] == "params"
        n = int(tok[i + 1])
        params = np.array([float(x) for x in tok[i + 2:i + 2 + n]], dtype=np.float32)
        sel = cls(n_hidden=h, margin=margin)
        sel.mu, sel.sd, sel.tmu = mu, sd, tmu
        sel.net.params = torch.tensor(params, dtype=torch.float32, device="cuda")
        return sel


DEFAULT_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "selector_mi355x_fp64.txt")


def heuristic_choice(kind: str, dim: int, degree: int) -> int:
    """The paper's complexity model (Sec. 4.4): T_Q / T_T ~ (2q + n_f q - n_D)^d (n_f + n_D d + 1)
    / (q^{n_f d} d^{n_D}); tensor representation (library default launch) when it predicts
    a speedup, else the quadrature kernel."""
    n_f = 1 if kind in ("wlaplace", "ns") else 0
    n_D = {"mass": 0, "laplace": 2, "wlaplace": 2, "elasticity": 2, "ns": 1}[kind]
    q = degree
    p = max(2 * q + n_f * q - n_D, 1)
    speedup = p ** dim * (n_f + n_D * dim + 1) / (q ** (n_f * dim) * dim ** n_D)
    return 0 if speedup > 1.0 else len(CANDIDATES_FP64) - 1


def regret(records, choices):
    """Per-record t_chosen / t_best - 1, with the exhaustive minimum as the judge."""
    out = []
    for r, c in zip(records, choices):
        valid = [t for t in r["ms"] if t is not None and t > 0]
        out.append(r["ms"][c] / min(valid) - 1.0)
    return np.array(out)


if __name__ == "__main__":
    import argparse

    from . import tune

    ap = argparse.ArgumentParser(description="train the selector on a stored sweep (on the GPU, with the "
                                             "library's own MLP kernels) and write the file FFC_KERNEL_AUTO reads")
    ap.add_argument("--sweep", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                                                    "sweep_mi355x_fp64.jsonl"))
    ap.add_argument("--out", default=DEFAULT_FILE)
    ap.add_argument("--epochs", type=int, default=3000)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    sel = Selector(seed=args.seed)
    loss = sel.fit(tune.load_sweep(args.sweep), epochs=args.epochs)
    sel.export(args.out)
    print(f"selector: trained on {args.sweep} (final loss {loss:.4f}), written to {args.out}", flush=True)
