"""Shared helpers for the parity tests (comparison metrics, case printing)."""
import sys

import numpy as np


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def announce(*what):
    """Names the case before a GPU step so a crash can be attributed."""
    print("CASE", *what, flush=True)
    sys.stdout.flush()


def positions(cfg, parts: dict) -> np.ndarray:
    """Global positions (3, N) reconstructed from cell index and offsets."""
    c = parts["cell"].astype(np.int64)
    ijk = [c % cfg.nx, (c // cfg.nx) % cfg.ny, c // (cfg.nx * cfg.ny)]
    offs = [parts["ox"], parts["oy"], parts.get("oz", np.zeros(c.size))]
    h = (cfg.dx, cfg.dy, cfg.dz)
    return np.stack([(ijk[a] + 0.5 + 0.5 * np.asarray(offs[a], np.float64)) * h[a]
                     for a in range(3)])


def compare_particles(cfg, gpu: dict, ref: dict, band=1e-5, vtol=2e-6):
    """Cell indices must agree bit-exactly except for particles the oracle puts
    within `band` (half-cell units) of a cell face ("straddlers"); those must
    agree in position.  Offsets and velocities agree to FP32 rounding."""
    offs = ["ox", "oy"] + (["oz"] if cfg.ndim == 3 else [])
    near = np.zeros(ref["cell"].size, bool)
    for k in offs:
        o = np.asarray(ref[k], np.float64)
        near |= (np.abs(o + 1.0) < band) | (np.abs(o - 1.0) < band)
    diff = gpu["cell"] != ref["cell"]
    assert not np.any(diff & ~near), f"{int(np.sum(diff & ~near))} cell mismatches off the faces"
    L = np.array([cfg.nx * cfg.dx, cfg.ny * cfg.dy, cfg.nz * cfg.dz])[:, None]
    d = positions(cfg, gpu) - positions(cfg, ref)
    d -= np.round(d / L) * L
    h = np.array([cfg.dx, cfg.dy, cfg.dz])[:, None]
    assert np.abs(d / h).max() < 1e-5, np.abs(d / h).max()
    same = ~diff
    for k in offs:
        assert np.abs(np.asarray(gpu[k], np.float64)[same] - ref[k][same]).max() < 1e-5
    vs = max(np.abs(ref[k]).max() for k in ("ux", "uy", "uz"))
    for k in ("ux", "uy", "uz"):
        err = np.abs(np.asarray(gpu[k], np.float64) - ref[k]).max()
        assert err <= vtol * vs, (k, err, vs)
    return int(np.sum(diff))
