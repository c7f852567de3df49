"""Helpers for the GPU parity tests: device transfer, error norms and the error model.

Every comparison with the FP64 oracle checks two figures against one bound:
  norm-wise   ||got - ref|| / ||ref|| over the whole field
  per site    max_s |got_s - ref_s| / max_s |ref_s|, with |.| the 2-norm of one site's
              12 components, so that a few sites that are far off cannot hide in a
              field-wide norm.
The bounds (TOL) follow the arithmetic of each path:
  f64   1e-13 for the operator and for SAP: reordered FP64 sums, unit roundoff 1.1e-16 times a
        few hundred terms (the MR steps of a few cycles keep SAP at the operator's level)
  f32   2e-6 for the operator and for SAP: FP32 storage and arithmetic, unit roundoff 6e-8
        times the square root of the ~100 terms of a site's result, about 6e-7, with room for
        the MR steps' coefficients (the kernels reach 2.4e-7 at most)
  f16   2e-3: links and spinors rounded to FP16 at every store (unit roundoff 2^-11 = 4.9e-4
        relative to the site's scale), about four roundings' worth
  bf16  1.5e-2: the same with BF16's unit roundoff 2^-8 = 3.9e-3
When TM_ERR_LOG names a file, each check appends its measured figures to it (one JSON object
per line), which is how the measured-error table of the design notes is produced.
"""
import json
import os

import numpy as np

TOL = {
    "dirac": {"f64": 1e-13, "f32": 2e-6, "f16": 2e-3, "bf16": 1.5e-2},
    "sap": {"f64": 1e-13, "f32": 2e-6, "f16": 2e-3, "bf16": 1.5e-2},
}


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    """Norm-wise relative error ||a - b|| / ||b||."""
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def site_err(a, b):
    """Per-site error max_s |a_s - b_s| / max_s |b_s| (12 complex components per site)."""
    a = np.asarray(a).reshape(-1, 12)
    b = np.asarray(b).reshape(-1, 12)
    return float(np.linalg.norm(a - b, axis=1).max() / np.linalg.norm(b, axis=1).max())


def log_error(record):
    path = os.environ.get("TM_ERR_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(record) + "\n")


def check_close(got, ref, kind, prec, label, tol=None):
    """Asserts both error figures of got against the FP64 reference below the bound TOL[kind][prec]."""
    bound = TOL[kind][prec] if tol is None else tol
    ne, se = rel_err(got, ref), site_err(got, ref)
    log_error({"kind": kind, "prec": prec, "case": label, "norm": ne, "site": se, "bound": bound})
    print(f"  {kind} {prec} {label}: norm-wise {ne:.2e}, per-site {se:.2e} (bound {bound:.0e})", flush=True)
    assert ne < bound, (label, "norm-wise", ne, bound)
    assert se < bound, (label, "per-site", se, bound)
    return ne, se


def log_solve(label, prec, oracle_rel, tol, iters=None):
    """Records a solve's true relative residual as recomputed by the oracle (the bound is tol)."""
    log_error({"kind": "solve", "prec": prec, "case": label, "norm": float(oracle_rel), "site": None, "bound": tol,
               "iters": iters})


def announce(msg):
    print(msg, flush=True)
