"""Completion-quality harness (Sec. 3.6 metrics on the held-out protocol of
Sec. 3.7): hold out a share of the observed cells, fit on the rest, and
measure RMSE-A (training cells), RMSE-P (held-out cells) and the distance
correlation of the held-out cells' original and approximated values.  The
fit and the metrics run on the GPU through the C ABI (stmf_fit,
stmf_completion_metrics); the split is a seeded input draw."""
from __future__ import annotations

import time

import numpy as np

from . import stmf, synth


def evaluate(R, M, rank, iters, seed=0, frac=0.2, split_seed=0, device="cuda", **opts):
    """R (float32), M (uint8): host arrays.  Returns the metrics, the fit's
    time, final training error and trial counts, and the split's sizes."""
    import torch
    M_train, M_test = synth.holdout(M, frac, split_seed)
    Rd = torch.from_numpy(np.ascontiguousarray(R, np.float32)).to(device)
    Mtr = torch.from_numpy(M_train).to(device)
    Mte = torch.from_numpy(M_test).to(device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fit = stmf.stmf_fit(Rd, Mtr, rank, iters, seed=seed, **opts)
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t0
    met = stmf.stmf_completion_metrics(Rd, Mtr, Mte, fit.U, fit.V)
    met.update(fit_s=fit_s, final_error=float(fit.traj[-1]), trials=fit.info["trials"],
               accepted=fit.info["accepted"], iters_done=fit.info["iters_done"])
    return met, fit, (M_train, M_test)
