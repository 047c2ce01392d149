"""Run-time tile-configuration choice: tuned database, then the learned model,
then the library's built-in default.

The paper fixes its tuning parameters per architecture at compile time (Sec. 2.3,
Sec. 3, Tab. 4) and names automatic tuning as the way forward (Sec. 6).  Here a
GEMM's configuration is chosen per call:

1. ``database`` -- the shape was timed by the tuner: its exhaustive best;
2. ``model``    -- otherwise the MLP cost model predicts one (evaluated by the
                   library's HIP kernels); with ``measure_top = k`` the k best
                   predicted configurations are run once each on operands of
                   the shape and the fastest is kept (``measured``);
3. ``default``  -- no model (or no GPU to evaluate it): the library's built-in
                   preference list (``cfg = None``).

Predictions are cached per (dtype, m, n, k)."""
from __future__ import annotations

import os

from . import F32, F64, Cfg, configs, gemm

DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


class ConfigChooser:
    def __init__(self, db_path: str | None = os.path.join(DATA, "tune_db.json.gz"),
                 model_path: str | None = os.path.join(DATA, "model.mlp"), measure_top: int = 0):
        from . import tune
        self.measure_top = measure_top
        self._best = {}
        if db_path and os.path.exists(db_path):
            db = tune.load_compact(db_path)
            valid = {dt: {c.as_tuple() for c in configs(dt)} for dt in (F64, F32)}
            top = {}
            for r in db.records:
                key = (r["dtype"], r["m"], r["n"], r["k"])
                c = tuple(r["cfg"])
                if r["dtype"] not in valid or c not in valid[r["dtype"]]:
                    continue                      # a configuration no longer registered
                if key not in top or r["tflops"] > top[key][1]:
                    top[key] = (c, r["tflops"])
            self._best = {k: v[0] for k, v in top.items()}
        self._model_path = model_path
        self._pred = None
        self._cache = {}

    def _model(self):
        if self._pred is None and self._model_path and os.path.exists(self._model_path):
            from . import learn
            self._pred = learn.Predictor.load(self._model_path, check_table=learn.config_table())
        return self._pred

    def choose(self, m: int, n: int, k: int, dtype: int = F64):
        """(Cfg or None, source) for an m x n x k GEMM of dtype F64 or F32."""
        key = (dtype, m, n, k)
        if key in self._best:
            return Cfg(*self._best[key]), "database"
        if key in self._cache:
            return self._cache[key]
        out = (None, "default")
        if dtype in (F64, F32) and min(m, n, k) >= 1:
            try:
                pred = self._model()
                import torch
                if pred is not None and torch.cuda.is_available():
                    from . import learn
                    if self.measure_top > 1:
                        out = (self._measured(pred, dtype, m, n, k), "measured")
                    else:
                        slot = learn.predict(pred, [(dtype, m, n, k)])[0]
                        out = (Cfg(*pred.table[slot][1]), "model")
            except (ImportError, ValueError, OSError):
                out = (None, "default")
        self._cache[key] = out
        return out

    def _measured(self, pred, dtype, m, n, k):
        """The fastest of the model's measure_top best predictions, each timed
        once (after one untimed run) on operands of the shape drawn for it."""
        from . import learn, tune
        slots = learn.ranked(pred, [(dtype, m, n, k)], self.measure_top)[0]
        ops = tune.Operands(m, n, k, dtype)
        best, best_t = None, None
        for j in slots:
            cfg = Cfg(*pred.table[j][1])
            t = min(tune.time_config(ops, dtype, cfg, warmup=1, reps=1))
            if best_t is None or t < best_t:
                best, best_t = cfg, t
        return best


_default = None


def tuned_gemm(A, B, C, alpha: float = 1.0, beta: float = 0.0, chooser: ConfigChooser | None = None,
               stream=None):
    """gemm() with the configuration chosen by ``chooser`` (a shared default
    chooser when None); returns (C, source)."""
    global _default
    if chooser is None:
        if _default is None:
            _default = ConfigChooser()
        chooser = _default
    from . import dtype_of
    dt = dtype_of(A)
    cfg, source = chooser.choose(A.shape[0], B.shape[1], A.shape[1], dt)
    gemm(A, B, C, alpha, beta, cfg=cfg, stream=stream)
    return C, source
