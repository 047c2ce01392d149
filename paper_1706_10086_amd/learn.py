"""Learned tile-configuration predictor on top of the autotuner's database.

The paper tunes its two parameters by exhaustive search on two matrix sizes
(Sec. 2.3, Sec. 3 Tab. 4) and concludes that more tuning parameters make tuning
itself expensive (Sec. 6).  Here the tuner's sweep over many shapes trains a
small network that predicts, for an unseen shape, the relative speed of every
configuration; the configuration with the highest prediction is used, and the
exhaustive sweep remains the fallback and the measure of the prediction's regret.

* features  x = [log2 m, log2 n, log2 k, dtype == F64, dtype == F32, w], w = 1
            where the rows of A and B are whole 16-byte loads (only then do the
            three-stage configurations run their own kernels; the tuner's shapes
            are stored without padding, lda = k, ldb = n), scaled by the training
            set's mean and standard deviation;
* targets   r_c^p with r_c = TFLOP/s(c) / max_c' TFLOP/s(c') for every
            configuration c of the shape's dtype (a masked multi-output
            regression; configurations of other dtypes are masked out); the power
            p (TARGET_POWER) leaves the arg-max unchanged and spends the fit on the
            configurations near the best, which are the ones the choice turns on;
* model     the library's MLP (6 -> 64 -> 64 -> V, FP32), trained by its own HIP
            kernels with Adam on the masked mean square error;
* choice    masked arg-max of the prediction;
* metrics   achieved fraction of the exhaustive best per held-out shape, with
            its geometric mean, median, 10th percentile and the share >= 0.95;
            the baseline without the model is the paper's method: one tuned
            configuration per dtype, the one with the best geometric-mean
            relative speed over the training shapes.
"""
from __future__ import annotations

import hashlib
import json
import math
from dataclasses import dataclass, field

import numpy as np

from . import F32, F64, MLP, configs

DTYPES = (F64, F32)


def config_table():
    """Output slots: (dtype, cfg tuple) for every registered configuration of the
    dtypes with a registry, in registry order."""
    table = []
    for dt in (F64, F32):
        for c in configs(dt):
            table.append((dt, c.as_tuple()))
    return table


def table_hash(table) -> str:
    return hashlib.sha1(json.dumps([[d, list(c)] for d, c in table]).encode()).hexdigest()[:12]


def rows_whole_loads(n, k, dtype, lda=None, ldb=None) -> bool:
    """Whether the rows of A (lda, default k) and B (ldb, default n) are whole
    16-byte loads: n, lda, ldb multiples of 2 (FP64) or 4 (FP32)."""
    epu = 4 if dtype == F32 else 2
    lda = k if lda is None else lda
    ldb = n if ldb is None else ldb
    return n % epu == 0 and lda % epu == 0 and ldb % epu == 0


def raw_features(m, n, k, dtype) -> np.ndarray:
    """Features of a product stored without padding (lda = k, ldb = n)."""
    oh = [1.0 if dtype == d else 0.0 for d in DTYPES]
    w = 1.0 if rows_whole_loads(n, k, dtype) else 0.0
    return np.array([math.log2(m), math.log2(n), math.log2(k)] + oh + [w], dtype=np.float64)


@dataclass
class Dataset:
    shapes: list            # (dtype, m, n, k)
    X: np.ndarray           # raw features
    T: np.ndarray           # relative speeds (0 where masked)
    M: np.ndarray           # mask
    tflops: np.ndarray      # measured TFLOP/s per slot (nan where not measured)


def build_dataset(db, table, shapes_with_dtype) -> Dataset:
    """Rows for every (dtype, m, n, k) that has measurements of all the dtype's
    slots in the database."""
    slot = {key: i for i, key in enumerate(table)}
    V = len(table)
    by_shape = {}
    for r in db.records:
        key = (r["dtype"], r["m"], r["n"], r["k"])
        by_shape.setdefault(key, {})[tuple(r["cfg"])] = max(
            r["tflops"], by_shape.get(key, {}).get(tuple(r["cfg"]), 0.0))
    shapes, X, T, M, TF = [], [], [], [], []
    for (dt, m, n, k) in shapes_with_dtype:
        meas = by_shape.get((dt, m, n, k))
        want = [c for (d, c) in table if d == dt]
        if not meas or any(c not in meas for c in want):
            continue
        tf = np.full(V, np.nan)
        for c in want:
            tf[slot[(dt, c)]] = meas[c]
        best = np.nanmax(tf)
        t = np.where(np.isnan(tf), 0.0, tf / best)
        mask = (~np.isnan(tf)).astype(np.float64)
        shapes.append((dt, m, n, k))
        X.append(raw_features(m, n, k, dt))
        T.append(t)
        M.append(mask)
        TF.append(tf)
    return Dataset(shapes, np.array(X), np.array(T), np.array(M), np.array(TF))


# ---------------------------------------------------------------------------
# The model file (the format mlp_save writes and mgemm_model_load reads; see
# csrc/model.hip): text, every floating-point value as a C99 hexadecimal float,
# closed by an FNV-1a checksum of the text before the checksum line.
# ---------------------------------------------------------------------------
def c_hex(x: float) -> str:
    """``x`` as glibc's printf("%a") writes a double (trailing zero digits of the
    fraction dropped), so that files written here and by the library agree."""
    mant, exp = float(x).hex().split("p")
    if "." in mant:
        mant = mant.rstrip("0").rstrip(".")
    return mant + "p" + exp


def fnv1a64(data: bytes) -> int:
    h = 0xcbf29ce484222325
    for b in data:
        h = ((h ^ b) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def model_text(table, mean, std, hidden, params) -> str:
    """The model file for a 6-input network with ``hidden`` units and one output
    per (dtype, configuration tuple) of ``table``."""
    params = np.asarray(params, dtype=np.float32)
    lines = ["mgemm-mlp 2", f"dims {len(mean)} {hidden} {len(table)}"]
    lines += ["out " + " ".join(str(int(v)) for v in (dt, *c)) for dt, c in table]
    lines.append("mean " + " ".join(c_hex(v) for v in mean))
    lines.append("std " + " ".join(c_hex(v) for v in std))
    lines.append(f"params {params.size}")
    vals = [c_hex(float(v)) for v in params]
    lines += [" ".join(vals[i:i + 8]) for i in range(0, len(vals), 8)]
    body = "\n".join(lines) + "\n"
    return body + f"checksum {fnv1a64(body.encode()):016x}\n"


def parse_model_text(text: str):
    """(table, mean, std, hidden, params) of a model file; ValueError if the
    checksum or the syntax is wrong."""
    cpos = text.rfind("checksum ")
    if cpos < 0 or (cpos > 0 and text[cpos - 1] != "\n"):
        raise ValueError("no checksum line")
    if int(text[cpos + 9:].split()[0], 16) != fnv1a64(text[:cpos].encode()):
        raise ValueError("checksum mismatch (corrupt file)")
    tok = text[:cpos].split()
    if tok[:2] != ["mgemm-mlp", "2"] or tok[2] != "dims":
        raise ValueError("not an mgemm-mlp version 2 file")
    I, H, O = (int(t) for t in tok[3:6])
    pos = 6
    table = []
    for _ in range(O):
        if tok[pos] != "out":
            raise ValueError("output line missing")
        v = [int(t) for t in tok[pos + 1:pos + 9]]
        table.append((v[0], tuple(v[1:])))
        pos += 9
    if tok[pos] != "mean":
        raise ValueError("no mean line")
    mean = np.array([float.fromhex(t) for t in tok[pos + 1:pos + 1 + I]])
    pos += 1 + I
    if tok[pos] != "std":
        raise ValueError("no std line")
    std = np.array([float.fromhex(t) for t in tok[pos + 1:pos + 1 + I]])
    pos += 1 + I
    if tok[pos] != "params":
        raise ValueError("no params line")
    P = int(tok[pos + 1])
    params = np.array([float.fromhex(t) for t in tok[pos + 2:pos + 2 + P]], dtype=np.float32)
    if params.size != P or pos + 2 + P != len(tok):
        raise ValueError("parameter count does not match")
    return table, mean, std, H, params


@dataclass
class Predictor:
    table: list
    mean: np.ndarray
    std: np.ndarray
    params: np.ndarray
    hidden: int = 64
    history: list = field(default_factory=list)

    def scaled(self, X):
        return (X - self.mean) / self.std

    def to_json(self) -> str:
        return json.dumps({"table": [[d, list(c)] for d, c in self.table],
                           "table_hash": table_hash(self.table), "mean": self.mean.tolist(),
                           "std": self.std.tolist(), "hidden": self.hidden,
                           "params": self.params.tolist(), "history": self.history})

    def save(self, path: str) -> None:
        """Writes the model file mgemm_model_load reads."""
        with open(path, "w") as f:
            f.write(model_text(self.table, self.mean, self.std, self.hidden, self.params))

    @classmethod
    def load(cls, path: str, check_table=None) -> "Predictor":
        """Reads a model file (ValueError if corrupt, or, with ``check_table``, if
        its outputs are not that table)."""
        with open(path) as f:
            table, mean, std, hidden, params = parse_model_text(f.read())
        if check_table is not None and table_hash(check_table) != table_hash(table):
            raise ValueError("model was trained for a different configuration table")
        return cls(table, mean, std, params, hidden)

    @classmethod
    def from_json(cls, s: str, check_table=None) -> "Predictor":
        d = json.loads(s)
        table = [(dt, tuple(c)) for dt, c in d["table"]]
        if table_hash(table) != d["table_hash"]:
            raise ValueError("corrupt model file (table hash)")
        if check_table is not None and table_hash(check_table) != d["table_hash"]:
            raise ValueError("model was trained for a different configuration table")
        return cls(table, np.array(d["mean"]), np.array(d["std"]), np.array(d["params"], dtype=np.float32),
                   d["hidden"], d.get("history", []))


TARGET_POWER = 4.0


def train(ds: Dataset, table, hidden=64, steps=4000, lr=2e-3, seed=5, log=None,
          power: float = TARGET_POWER, final_steps: int = 0, final_lr: float | None = None
          ) -> Predictor:
    """Fits the MLP on the GPU with the library's kernels (full-batch Adam):
    ``steps`` steps at ``lr``, then ``final_steps`` more at ``final_lr``."""
    import torch
    mean = ds.X.mean(axis=0)
    std = ds.X.std(axis=0)
    std[std == 0] = 1.0
    I, O = ds.X.shape[1], len(table)
    init = _init_params(I, hidden, O, seed)
    net = MLP(I, hidden, O, init)
    dev = torch.device("cuda")
    Xs = torch.from_numpy(((ds.X - mean) / std).astype(np.float32)).to(dev)
    net.set_data(Xs, torch.from_numpy((ds.T ** power).astype(np.float32)).to(dev),
                 torch.from_numpy(ds.M.astype(np.float32)).to(dev))
    hist = []
    done = 0
    chunk = 500
    for n_steps, rate in ((steps, lr), (final_steps, final_lr)):
        end = done + n_steps
        while done < end:
            s = min(chunk, end - done)
            loss = net.train(s, lr=rate)
            done += s
            hist.append((done, float(loss)))
            if log:
                log(f"  mlp step {done}: loss {loss:.5f}")
    params = net.get_params()
    net.destroy()
    return Predictor(table, mean, std, params, hidden, hist)


def _init_params(I, H, O, seed):
    """He-uniform weights from the seeded generator, zero biases (the same
    recipe as the oracle's he_uniform_init, restated here so the product path
    does not import the oracle)."""
    import synth
    parts = []
    for li, (fo, fi) in enumerate([(H, I), (H, H), (O, H)]):
        lim = np.sqrt(6.0 / fi)
        parts.append((synth.uniform_pm1((fo, fi), seed + li) * lim).ravel())
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


def predict(pred: Predictor, shapes_with_dtype) -> list:
    """Predicted slot index per (dtype, m, n, k), by the library's GPU kernels."""
    import torch
    X = np.array([raw_features(m, n, k, dt) for (dt, m, n, k) in shapes_with_dtype])
    M = np.array([[1.0 if d == dt else 0.0 for (d, _) in pred.table]
                  for (dt, _, _, _) in shapes_with_dtype])
    I, O = X.shape[1], len(pred.table)
    net = MLP(I, pred.hidden, O, pred.params)
    dev = torch.device("cuda")
    idx = net.predict(torch.from_numpy(pred.scaled(X).astype(np.float32)).to(dev),
                      torch.from_numpy(M.astype(np.float32)).to(dev)).cpu().numpy()
    net.destroy()
    return [int(i) for i in idx]


def ranked(pred: Predictor, shapes_with_dtype, k: int = 3) -> list:
    """The ``k`` slots with the highest predictions of each shape's dtype, best
    first (the network evaluated by the library's GPU kernels)."""
    import torch
    X = np.array([raw_features(m, n, kk, dt) for (dt, m, n, kk) in shapes_with_dtype])
    I, O = X.shape[1], len(pred.table)
    net = MLP(I, pred.hidden, O, pred.params)
    try:
        Y = net.forward(torch.from_numpy(pred.scaled(X).astype(np.float32)).cuda()).cpu().numpy()
    finally:
        net.destroy()
    out = []
    for (dt, _, _, _), y in zip(shapes_with_dtype, Y):
        allowed = [j for j, (d, _) in enumerate(pred.table) if d == dt]
        out.append(sorted(allowed, key=lambda j: -y[j])[:k])
    return out


def single_best_baseline(ds: Dataset, table) -> dict:
    """Per dtype: the slot with the best geometric-mean relative speed over the
    dataset (one tuned configuration per dtype, the paper's tuning outcome)."""
    out = {}
    for dt in {s[0] for s in ds.shapes}:
        rows = [i for i, s in enumerate(ds.shapes) if s[0] == dt]
        slots = [j for j, (d, _) in enumerate(table) if d == dt]
        logs = {j: np.mean(np.log(np.maximum(ds.T[rows, j], 1e-9))) for j in slots}
        out[dt] = max(logs, key=logs.get)
    return out


def achieved(ds: Dataset, choice) -> np.ndarray:
    """Fraction of the exhaustive best reached by the chosen slot per row."""
    return np.array([ds.T[i, c] for i, c in enumerate(choice)])


def summarize(frac: np.ndarray) -> dict:
    frac = np.asarray(frac, dtype=np.float64)
    return {"geomean": float(np.exp(np.mean(np.log(np.maximum(frac, 1e-9))))),
            "median": float(np.median(frac)), "p10": float(np.percentile(frac, 10)),
            "share_ge_0.95": float(np.mean(frac >= 0.95)), "n": int(frac.size)}


def top_k_fallback(ds: Dataset, pred: Predictor, k=3) -> np.ndarray:
    """Achieved fraction when the k best-predicted slots are measured and the
    fastest is kept (uses the database's measurements of those slots)."""
    import torch
    I, O = ds.X.shape[1], len(pred.table)
    net = MLP(I, pred.hidden, O, pred.params)
    Y = net.forward(torch.from_numpy(pred.scaled(ds.X).astype(np.float32)).cuda()).cpu().numpy()
    net.destroy()
    Y = np.where(ds.M > 0, Y, -np.inf)
    top = np.argsort(-Y, axis=1)[:, :k]
    return np.array([max(ds.T[i, j] for j in top[i] if ds.M[i, j] > 0) for i in range(len(top))])


# Training settings of the shipped model (paper_1706_10086_amd/data/model.mlp):
# 8000 Adam steps at 3e-3, 4000 more at 1e-3, targets r^4, seed 5.
TRAIN_SETTINGS = dict(steps=8000, lr=3e-3, final_steps=4000, final_lr=1e-3)
# The tuner's shape sets the model trains on (FP64 and FP32 each): the 3000
# 'train' and 3000 'train2' shapes and the 800 'aligned' ones (the same law,
# dimensions rounded up to multiples of 4, which the random draws rarely give);
# the 500 'heldout' shapes stay out and score it.
TRAIN_SETS = ("train", "train2", "aligned")


def datasets(db, table):
    """(training rows, held-out rows) of ``db`` for ``table``: FP64 and FP32 on
    the TRAIN_SETS shapes and on the held-out shapes."""
    from . import tune
    tr = [(dt, *s) for dt in (F64, F32) for name in TRAIN_SETS for s in tune.shape_set(name)]
    ho = [(dt, *s) for dt in (F64, F32) for s in tune.shape_set("heldout")]
    return build_dataset(db, table, tr), build_dataset(db, table, ho)


def main(argv=None):
    """Trains the predictor on a tuner database (the compact .json.gz form or a
    JSONL database) with the library's kernels and writes the model file that
    mgemm_model_load and the chooser read; prints the held-out scores."""
    import argparse
    from . import tune
    ap = argparse.ArgumentParser(description="train the tile-configuration predictor")
    ap.add_argument("--db", required=True)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    db = tune.load_compact(a.db) if a.db.endswith(".gz") else tune.DB.load(a.db)
    table = config_table()
    dtr, dho = datasets(db, table)
    if not dtr.shapes:
        raise SystemExit("the database has no training rows for the registered configurations")
    pred = train(dtr, table, log=lambda s: print(s, flush=True), **TRAIN_SETTINGS)
    pred.save(a.out)
    print(f"learn: wrote {a.out} ({len(dtr.shapes)} training rows, {len(table)} outputs)", flush=True)
    if dho.shapes:
        base = single_best_baseline(dtr, table)
        print("held-out, model:", summarize(achieved(dho, predict(pred, dho.shapes))), flush=True)
        print("held-out, one configuration per dtype:",
              summarize(achieved(dho, [base[s[0]] for s in dho.shapes])), flush=True)


if __name__ == "__main__":
    main()
