"""The seeded input recipes hold what their docstrings state (host only)."""
import numpy as np

from paper_2305_05600_amd import workloads as W


def test_ensemble_specs_ranges_and_seed():
    sp = W.ensemble_specs()
    assert len(sp) == 64
    assert sp == W.ensemble_specs()  # deterministic for a seed
    assert sp != W.ensemble_specs(seed=5)
    for s in sp:
        assert 64 <= s["side"] <= 256 and 32 <= s["ppc"] <= 200
        assert 0.001 <= s["amp"] <= 0.05 and 0.1 <= s["te_ratio"] <= 1.0
    total = sum(s["side"] ** 2 * s["ppc"] for s in sp)
    assert 150e6 < total < 300e6  # about 213M expected over seeds


def test_ensemble_run_follows_its_spec():
    s = dict(seed=3, side=12, ppc=21, amp=0.02, te_ratio=0.4, vth=0.5)
    cfg, parts, B = W.ensemble_run(s)
    assert (cfg.nx, cfg.ny, cfg.ndim) == (12, 12, 2)
    assert parts["cell"].size == 12 * 12 * 21
    assert np.bincount(parts["cell"], minlength=cfg.ncell).tolist() == [21] * cfg.ncell
    assert abs(cfg.te - 0.4 * 0.25) < 1e-12
    assert abs(float(np.abs(B[1]).max()) - 0.02) < 1e-3 and np.all(B[0] == 1.0)
