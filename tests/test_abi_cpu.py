"""Host-side checks of libhvpic.so that need no GPU: the library loads, exports
every function include/hvpic.h declares, and rejects bad arguments before any
device work (parameter validation is pure host code)."""
import ctypes
import pathlib
import re

import pytest

from paper_2305_05600_amd import workloads as W

ROOT = pathlib.Path(__file__).resolve().parents[1]


@pytest.fixture(scope="module")
def H():
    from paper_2305_05600_amd import hvpic

    if not hvpic.LIB_PATH.exists():
        from paper_2305_05600_amd import build

        build.build()
    hvpic.lib()
    return hvpic


def _declared():
    text = (ROOT / "include" / "hvpic.h").read_text()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(hvpic_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol(H):
    names = _declared()
    assert len(names) >= 10, names
    for n in names:
        assert hasattr(H.lib(), n), n
    assert set(names) == set(H.EXPORTS)


def test_struct_layout_matches_header(H):
    # hvpic_params: 4 int32, 4 double, 3 int32 (+pad), 8 double, int32 (+pad),
    # double, 2 int32, double, int64
    assert ctypes.sizeof(H.HvpicParams) == 16 + 32 + 16 + 64 + 16 + 8 + 8 + 8
    assert ctypes.sizeof(H.HvpicInflow) == 5 * 8 + 8
    text = (ROOT / "include" / "hvpic.h").read_text()
    body = text[text.index("typedef struct {"):text.index("} hvpic_params;")]
    fields = re.findall(r"(?:int32_t|int64_t|double)\s+([\w, ]+);", body)
    names = [n.strip() for f in fields for n in f.split(",")]
    assert names == [f[0] for f in H.HvpicParams._fields_]
    assert ctypes.sizeof(H.HvpicParticles) == 8 * 9


def test_workspace_bytes_and_validation(H):
    cfg, _, _ = W.periodic_alfven()
    p = H.params_from(cfg, 65536)
    nb = H.hvpic_workspace_bytes(p)
    assert nb > 65536 * 16
    bad = [dict(ndim=4), dict(nz=2), dict(dx=0.0), dict(dt=float("nan")), dict(shape=7),
           dict(n_floor=0.0), dict(eta_h=-1e-3), dict(eta_h=float("nan")),
           dict(energy_eq=2), dict(energy_eq=1, gamma_e=1.0), dict(energy_eq=1, gamma_e=0.5),
           dict(kappa0=-0.1), dict(kappa0=float("inf")), dict(np_capacity=-1), dict(nsub=-1),
           dict(open_x=2), dict(open_x=1, nx=2),
           dict(buffer_cells=-1), dict(eta_h_buffer=-0.1), dict(eta_h_buffer=float("nan"))]
    for b in bad:
        q = H.params_from(cfg, 65536)
        for k, v in b.items():
            setattr(q, k, v)
        n = ctypes.c_size_t(0)
        assert H.lib().hvpic_workspace_bytes(ctypes.byref(q), ctypes.byref(n)) == H.HVPIC_EINVAL, b
    for good in (dict(eta_h=1e-3), dict(energy_eq=1, gamma_e=5.0 / 3.0, kappa0=0.1),
                 dict(open_x=1, buffer_cells=4, eta_h_buffer=0.02)):
        q = H.params_from(cfg, 65536)
        for k, v in good.items():
            setattr(q, k, v)
        # open x adds the injection's per-row counts, offsets and slots
        extra = -(-3 * 2 * cfg.ny * 4 // 256) * 256 if good.get("open_x") else 0
        assert H.hvpic_workspace_bytes(q) == nb + extra, good
    # in 3D a face has ny nz rows
    q3 = H.params_from(cfg, 65536)
    q3.ndim, q3.nz = 3, 5
    nb3 = H.hvpic_workspace_bytes(q3)
    q3.open_x = 1
    assert H.hvpic_workspace_bytes(q3) == nb3 + -(-3 * 2 * cfg.ny * 5 * 4 // 256) * 256


def test_init_rejects_bad_arguments_without_device_work(H):
    cfg, _, _ = W.periodic_alfven()
    p = H.params_from(cfg, 10)
    ctx = ctypes.c_void_p()
    L = H.lib()
    assert L.hvpic_init(ctypes.byref(p), None, None, ctypes.byref(ctx)) == H.HVPIC_EINVAL
    assert L.hvpic_init(ctypes.byref(p), None, ctypes.c_void_p(0x1001), ctypes.byref(ctx)) \
        == H.HVPIC_EINVAL  # misaligned workspace
    assert L.hvpic_gather_push(None, None, None, None, None, None, None, None) == H.HVPIC_ESTATE
    assert L.hvpic_sort(None, None, None, None, None, 0) == H.HVPIC_ESTATE
    assert L.hvpic_sort_perm(None, None, None, None, None) == H.HVPIC_ESTATE
    assert L.hvpic_gather_push_perm(None, None, None, None, None, None, None, None, None,
                                    None) == H.HVPIC_ESTATE
    assert L.hvpic_finalize(None) == H.HVPIC_ESTATE
    assert L.hvpic_field_advance_pe(None, None, None, None, None, None, None, None, 0,
                                    None) == H.HVPIC_ESTATE
    assert L.hvpic_eos_pressure(None, None, None) == H.HVPIC_ESTATE
    assert L.hvpic_open_fill(None, None, 3) == H.HVPIC_ESTATE
    assert L.hvpic_open_field_advance(None, None, None, None, None, None, None, None, None, 0,
                                      None) == H.HVPIC_ESTATE
    assert L.hvpic_open_particles(None, None, None, 0, 0) == H.HVPIC_ESTATE
    assert L.hvpic_sort_open(None, None, None, None) == H.HVPIC_ESTATE
    assert H.hvpic_strerror(H.HVPIC_EINVAL) == "invalid argument"
    assert L.hvpic_set_stream(None, None) == H.HVPIC_ESTATE
    assert L.hvpic_timing_enable(None, 4, 1) == H.HVPIC_ESTATE
    d, k = ctypes.c_double(), ctypes.c_int64()
    assert L.hvpic_timing_read(None, 0, ctypes.byref(d), ctypes.byref(k)) == H.HVPIC_ESTATE
