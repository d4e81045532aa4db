"""Helpers of the GPU parity tests: run the library on a packed batch and compare with the oracle
using the per-output statistics of the tolerance definition (see ``errors``) and a tie-aware argmax
agreement."""
from __future__ import annotations

from typing import Dict

import numpy as np

TOL = {"fp32": 1e-5, "bf16": 2e-2}


def run_gpu(model, pk, prim: bool = False) -> Dict[str, np.ndarray]:
    import torch
    from paper_2601_17554_amd import binding as B

    x = torch.from_numpy(pk.x).cuda()
    batch = B.Batch.from_host(pk.row_start, pk.n_valid)
    p = torch.from_numpy(pk.prim).cuda() if prim else None
    out = model.reconstruct(x, batch, prim=p)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def errors(got: Dict[str, np.ndarray], ref: Dict[str, np.ndarray]) -> Dict[str, float]:
    """Errors of one event (rows already selected), in the form each output's tolerance uses:
      logits  : max |d logits| / max |logits|                  (max-abs, relative to the output)
      pt, e   : max |pT/pT_ref - 1|, max |E/E_ref - 1|         (relative on the decoded quantity;
                both are regressed as log-ratios, Eq. 2, so this is exp(d log) - 1)
      angles  : max |d (eta, sin, cos)| / max |regression outputs|   (max-abs over the block)
    Per-column norm-wise values are returned too (diag_*) for reporting."""
    e = {}
    lg, lr = got["logits"].astype(np.float64), ref["logits"]
    e["logits"] = np.abs(lg - lr).max() / max(np.abs(lr).max(), 1e-6)
    g, r = got["reg"].astype(np.float64), ref["reg"]
    e["pt"] = np.abs(np.expm1(g[:, 0] - r[:, 0])).max()
    e["energy"] = np.abs(np.expm1(g[:, 4] - r[:, 4])).max()
    e["angles"] = np.abs(g[:, 1:4] - r[:, 1:4]).max() / max(np.abs(r).max(), 1e-6)
    for c, name in enumerate(["pt", "eta", "sin", "cos", "e"]):
        e["diag_" + name] = np.abs(g[:, c] - r[:, c]).max() / max(np.abs(r[:, c]).max(), 1e-6)
    return e


def argmax_agreement(got_cls: np.ndarray, ref_logits: np.ndarray, tol: float):
    """(agreement over elements whose oracle top-1/top-2 margin exceeds 2*tol*||logits||_inf,
    raw agreement, fraction of near-ties)."""
    ref_cls = np.argmax(ref_logits, axis=1)
    srt = np.sort(ref_logits, axis=1)
    margin = srt[:, -1] - srt[:, -2]
    clear = margin > 2 * tol * max(np.abs(ref_logits).max(), 1e-6)
    raw = float((got_cls == ref_cls).mean()) if len(ref_cls) else 1.0
    agree = float((got_cls[clear] == ref_cls[clear]).mean()) if clear.any() else 1.0
    return agree, raw, 1.0 - float(clear.mean()) if len(clear) else 0.0


def check_event(got_all, ref, rows, tol: float, label: str = ""):
    got = {k: v[rows] for k, v in got_all.items()}
    e = errors(got, ref)
    print(f"{label}: " + ", ".join(f"{k} {v:.2e}" for k, v in e.items() if not k.startswith("diag_")),
          flush=True)
    bad = {k: v for k, v in e.items() if not k.startswith("diag_") and not v <= tol}
    assert not bad, f"{label}: errors above {tol}: {bad} (all: {e})"
    agree, raw, ties = argmax_agreement(got["cls"], ref["logits"], tol)
    assert agree >= 0.999, f"{label}: argmax agreement {agree} (raw {raw}, near-ties {ties})"
    return e
