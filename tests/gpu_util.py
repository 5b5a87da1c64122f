"""Helpers shared by the GPU tests: run the HIP path through the C ABI on a
seeded workload and return numpy arrays.  Nothing here computes any part of
the method."""
import numpy as np
import torch

from paper_2004_12484_amd import enuf


def to_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def run(x, q, box, alpha, rc, M, p, precision="f64", potential=True, forces=True, ke=1.0, eng=None):
    """One evaluation; returns (engine, dict of numpy results)."""
    if eng is None:
        eng = enuf.Enuf(box, len(q), alpha, rc, M, p, precision=precision, ke=ke)
    dt = eng.dtype
    xt = to_dev(x, dt)
    qt = to_dev(q, dt)
    E, F, phi = eng.energy_forces(xt, qt, forces=forces, potential=potential)
    torch.cuda.synchronize()
    out = {"E": E.cpu().numpy()}
    if F is not None:
        out["F"] = F.double().cpu().numpy()
    if phi is not None:
        out["phi"] = phi.double().cpu().numpy()
    out["_x"], out["_q"] = xt, qt
    return eng, out


def rms_rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
