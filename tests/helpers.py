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


def _near_face(o, band):
    o = np.asarray(o, np.float64)
    return (np.abs(o + 1.0) < band) | (np.abs(o - 1.0) < band)


def deposit_point_straddlers(cfg, parts: dict, back: float, band=1e-5) -> np.ndarray:
    """Particles whose deposit point x - back*v lies within `band` half-cells of
    a cell face (FP64).  FP32 and FP64 may put such a point in different cells."""
    offs = [("ox", "ux", cfg.dx), ("oy", "uy", cfg.dy)] + ([("oz", "uz", cfg.dz)] if cfg.ndim == 3 else [])
    bad = np.zeros(parts["cell"].size, bool)
    for ko, kv, h in offs:
        x = np.asarray(parts[ko], np.float64) - 2.0 * back * np.asarray(parts[kv], np.float64) / h
        x = x - 2.0 * np.floor((x + 1.0) / 2.0)
        bad |= _near_face(x, band)
    return bad


def drop_straddlers(cfg, parts: dict, B, steps: int = 1, band=1e-5, fused=False) -> dict:
    """Removes from the input every particle that the FP64 oracle moves, within
    `steps` steps, to within `band` half-cells of a face, or whose mid-point
    deposit point lands there.  Uses only the oracle (with the step's
    smoothing passes, if any); the GPU and the oracle then run on the same
    cleaned input, so cell decisions can be compared exactly (the straddler
    band of the parity contract).  Prints how many were removed."""
    import oracle as O

    keep = np.ones(parts["cell"].size, bool)
    for _ in range(4):
        sub = {k: v[keep] for k, v in parts.items()}
        ids = np.nonzero(keep)[0]
        sim = O.OracleSim(cfg, {**sub, "id": ids.astype(np.float64)}, B)
        bad = np.zeros(parts["cell"].size, bool)
        for _ in range(steps):
            E, Bg = sim.E, sim.B
            if cfg.nsmooth:
                E, Bg = O.smooth(cfg, E, cfg.nsmooth), O.smooth(cfg, Bg, cfg.nsmooth)
            O.push(cfg, sim.p, E, Bg)
            offs = ["ox", "oy"] + (["oz"] if cfg.ndim == 3 else [])
            near = np.zeros(sim.p["cell"].size, bool)
            for k in offs:
                near |= _near_face(sim.p[k], band)
            near |= deposit_point_straddlers(cfg, sim.p, 0.5 * cfg.dt, band)
            bad[sim.p["id"].astype(np.int64)[near]] = True
            perm, sim.cell_start = O.sort(cfg, sim.p["cell"])
            sim.p = O.apply_perm(sim.p, perm)
            n_half, J_half = O.deposit(cfg, sim.p, 0.5 * cfg.dt)
            if cfg.nsmooth:
                n_half = O.smooth(cfg, n_half, cfg.nsmooth)
                J_half = O.smooth(cfg, J_half, cfg.nsmooth)
            sim._advance(n_half, J_half, sim.n_prev, sim.J_prev, mode=0)
            sim.n_prev, sim.J_prev = n_half, J_half
        if not bad.any():
            print(f"straddlers removed: {int((~keep).sum())} of {keep.size} "
                  f"(band {band:g} half-cells, {steps} step(s))", flush=True)
            return {k: np.ascontiguousarray(v) for k, v in sub.items()}
        keep &= ~bad
    raise AssertionError("straddler removal did not converge")


def drop_push_straddlers(cfg, parts: dict, E, B, back=None, band=1e-5) -> dict:
    """For one push in the given fields: removes the particles that the FP64
    oracle puts within `band` half-cells of a face, and (back given) whose
    deposit point x - back v lands there.  Prints how many were removed."""
    import oracle as O

    ref = O.particles64(parts)
    O.push(cfg, ref, E, B)
    near = np.zeros(ref["cell"].size, bool)
    for k in ["ox", "oy"] + (["oz"] if cfg.ndim == 3 else []):
        near |= _near_face(ref[k], band)
    if back is not None:
        near |= deposit_point_straddlers(cfg, ref, back, band)
    print(f"straddlers removed: {int(near.sum())} of {near.size}", flush=True)
    return {k: np.ascontiguousarray(v[~near]) for k, v in parts.items()}


def check_field_diag(got, ref, tol=1e-5, we_bound=None):
    """The field diagnostics {W_B, W_dB, W_e} against the oracle to the accuracy
    that the field contract (tol relative L2 on B and n) implies:
      W_B within 2 tol relative (|dW_B| <= |B| |dB| V);
      W_dB within 2 tol sqrt(W_dB W_B) absolute: the error of the fluctuation
        energy is bounded by |B - <B>| |dB| V with |dB| <= tol |B|, so a
        fluctuation far below the mean field (B0 + a small dB stored in FP32)
        is known only to that absolute accuracy;
      W_e within tol relative, or within we_bound (absolute) when given: for
        a density near n0 the isothermal W_e = T_e V sum n ln(n/n0) is a sum
        of cancelling terms, and what the contract on n fixes is the bound
        of electron_energy_bound."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    print(f"field diagnostics gpu {got} oracle {ref}", flush=True)
    assert abs(got[0] - ref[0]) <= 2 * tol * abs(ref[0]), (got, ref)
    assert abs(got[1] - ref[1]) <= 2 * tol * np.sqrt(abs(ref[1] * ref[0])), (got, ref)
    lim = tol * abs(ref[2]) if we_bound is None else max(tol * abs(ref[2]), we_bound)
    assert abs(got[2] - ref[2]) <= lim, (got, ref, lim)


def check_push_diag(got, ref, cfg, parts: dict, tol=1e-5):
    """The push diagnostics {K, P} against the oracle: K within tol relative
    (a sum of positive terms); each component of P within tol sum m w |v|
    over the pushed ions `parts` (the oracle's): the velocity contract is
    relative to the speeds, and a drift-free component of P is a sum of
    cancelling terms."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = cfg.ms * float(np.sum(np.asarray(parts["w"], np.float64) * np.sqrt(
        sum(np.asarray(parts[k], np.float64) ** 2 for k in ("ux", "uy", "uz")))))
    print(f"push diagnostics gpu {got} oracle {ref} (P scale {scale:.4g})", flush=True)
    assert abs(got[0] - ref[0]) <= tol * abs(ref[0]), (got, ref)
    assert np.all(np.abs(got[1:] - ref[1:]) <= tol * scale), (got, ref, scale)


def electron_energy_bound(cfg, n, tol=1e-5, mask=None) -> float:
    """The largest change of W_e that a density error of relative L2 norm
    tol can make, to first order (Cauchy-Schwarz): ||dW_e/dn||_2 tol ||n||_2.
    dW_e/dn per cell is T_e V (1 + ln(n_f/n0)) for gamma = 1 and
    n0 T_e V gamma/(gamma - 1) (n_f/n0)^(gamma-1) / n0 otherwise (n_f the
    floored density; cells below the floor do not respond).  mask selects
    the cells W_e sums over."""
    n = np.asarray(n, np.float64).ravel()
    if mask is not None:
        n = n[np.asarray(mask).ravel()]
    nf = np.maximum(n, cfg.n_floor)
    V = cfg.dx * cfg.dy * cfg.dz
    if cfg.gamma_e == 1.0:
        d = cfg.te * V * (1.0 + np.log(nf / cfg.n0))
    else:
        d = cfg.te * V * cfg.gamma_e / (cfg.gamma_e - 1.0) * (nf / cfg.n0) ** (cfg.gamma_e - 1.0)
    d = np.where(n >= cfg.n_floor, d, 0.0)
    return float(np.linalg.norm(d) * tol * np.linalg.norm(n))


def drop_open_straddlers(cfg, parts: dict, B0, B1, spec: dict, seed: int, band=1e-5) -> dict:
    """For the first step of an open run (oracle.OpenOracleSim): removes
    the ions that the FP64 oracle's push puts within `band` half-cells of a
    face, or whose mid-point deposit point lands there.  Uses only the
    oracle; prints how many were removed."""
    import oracle as O

    keep = np.ones(parts["cell"].size, bool)
    for _ in range(4):
        sub = {k: v[keep] for k, v in parts.items()}
        sim = O.OpenOracleSim(cfg, sub, B0, B1, spec, seed)
        ids = np.nonzero(keep)[0]
        p = O.particles64({**sub, "id": ids.astype(np.float64)})
        perm, _ = O.sort(cfg, p["cell"])
        p = O.apply_perm(p, perm)
        O.push(cfg, p, sim.E, sim.Btot)
        near = _near_face(p["ox"], band) | _near_face(p["oy"], band)
        if cfg.ndim == 3:
            near |= _near_face(p["oz"], band)
        near |= deposit_point_straddlers(cfg, p, 0.5 * cfg.dt, band)
        if not near.any():
            print(f"straddlers removed: {int((~keep).sum())} of {keep.size} "
                  f"(band {band:g} half-cells, 1 open step)", flush=True)
            return {k: np.ascontiguousarray(v) for k, v in sub.items()}
        keep[p["id"].astype(np.int64)[near]] = False
    raise AssertionError("straddler removal did not converge")
