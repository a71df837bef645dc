"""Host-side checks of the C-ABI library: it loads without a GPU, exports
every entry point the public header declares, and rejects bad arguments
with the documented codes before touching the device."""
import ctypes
import os
import re

import pytest

import paper_1211_4864_amd as hsr
from paper_1211_4864_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hacc_sr.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hsr.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return hsr.load()


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hacc_sr_\w+)\s*\(", src)))


def test_header_declarations_are_exported(lib):
    names = declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(names) == sorted(_lib.EXPORTS)


def test_version_and_strerror(lib):
    assert lib.hacc_sr_version() >= 100
    for code in (0, -1, -2, -3, -4):
        assert len(hsr.strerror(code)) > 0


def test_grid_and_workspace_sizes(lib):
    assert hsr.grid_dim(1.0, 3 / 256) == 85
    assert hsr.grid_dim(1.0, 3 / 128) == 42
    assert hsr.grid_dim(-(1 + 6 / 512), 3 / 512) == 172
    assert hsr.workspace_bytes(256 ** 3, 1.0, 3 / 256) > 48 * 256 ** 3
    with pytest.raises(hsr.HaccSrError) as e:
        hsr.grid_dim(1.0, 0.4)                 # periodic box below 3 r_cut
    assert e.value.code == -2


P = ctypes.c_void_p
F = ctypes.c_float


def _poly(vals=(0,) * 6):
    return _lib.poly_array(vals)


@pytest.mark.parametrize("args,code", [
    ((None, None, -1, 1.0, F(0.1), F(1e-5)), -1),          # n < 0
    ((None, None, 10, 1.0, F(0.1), F(1e-5)), -1),          # null pointers
    ((P(16), P(16), 10, 1.0, F(0.0), F(1e-5)), -1),        # r_cut <= 0
    ((P(16), P(16), 10, 1.0, F(0.1), F(0.0)), -1),         # eps <= 0
    ((P(16), P(16), 10, float("nan"), F(0.1), F(1e-5)), -1),
    ((P(16), P(16), 10, 0.0, F(0.1), F(1e-5)), -1),        # box == 0
    ((P(16), P(16), 10, 1.0, F(0.5), F(1e-5)), -2),        # box < 3 r_cut
    ((P(16), P(16), 2 ** 31, 1.0, F(0.1), F(1e-5)), -2),   # n >= 2^31
    ((P(16), P(16), 10, 1.0, F(1e-4), F(1e-5)), -2),       # too many cells
    ((P(16), P(16), 1_200_000_000, 1.0, F(7.76e-4), F(1e-5)), -2),  # work items >= 2^31
])
def test_force_argument_validation(lib, args, code):
    assert lib.hacc_sr_set_workspace(None, 0) == 0
    rc = lib.hacc_sr_force(*args, _poly(), P(16))
    assert rc == code


def test_nonfinite_poly_and_missing_workspace(lib):
    assert lib.hacc_sr_set_workspace(None, 0) == 0
    bad = _poly((1.0, float("inf"), 0, 0, 0, 0))
    assert lib.hacc_sr_force(P(16), P(16), 10, 1.0, F(0.1), F(1e-5), bad, P(16)) == -1
    # valid arguments but no workspace registered
    assert lib.hacc_sr_force(P(16), P(16), 10, 1.0, F(0.1), F(1e-5), _poly(), P(16)) == -3
    assert lib.hacc_sr_force_vjp(P(16), P(16), 10, 1.0, F(0.1), F(1e-5), _poly(),
                                 P(16), P(16)) == -3
    assert lib.hacc_sr_bin(P(16), P(16), 10, 1.0, F(0.1), P(16), P(16), P(16)) == -3
    # a workspace that is too small
    assert lib.hacc_sr_set_workspace(P(256), 1024) == 0
    assert lib.hacc_sr_force(P(16), P(16), 10, 1.0, F(0.1), F(1e-5), _poly(), P(16)) == -3
    assert lib.hacc_sr_set_workspace(None, 0) == 0


def test_zero_particles_is_a_noop(lib):
    assert lib.hacc_sr_force(None, None, 0, 1.0, F(0.1), F(1e-5), _poly(), None) == 0
    assert lib.hacc_sr_force_vjp(None, None, 0, 1.0, F(0.1), F(1e-5), _poly(),
                                 None, None) == 0
    assert lib.hacc_sr_kick(None, None, 0, 0.1) == 0
    assert lib.hacc_sr_stream(None, None, 0, 0.1, 1.0) == 0
    assert lib.hacc_sr_kick_adjoint(None, None, 0, 0.1) == 0


def test_integrator_argument_validation(lib):
    assert lib.hacc_sr_kick(None, None, 5, 0.1) == -1
    assert lib.hacc_sr_kick(P(16), P(16), -1, 0.1) == -1
    assert lib.hacc_sr_kick(P(16), P(16), 5, float("inf")) == -1
    assert lib.hacc_sr_stream(P(16), P(16), 5, 0.1, float("nan")) == -1
    assert lib.hacc_sr_kick_adjoint(P(16), None, 5, 0.1) == -1
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    assert lib.hacc_sr_timing_read(8, ctypes.byref(n), ctypes.byref(ms)) == -1
    assert lib.hacc_sr_timing_read(-1, ctypes.byref(n), ctypes.byref(ms)) == -1


def test_product_path_has_no_fallback(monkeypatch, tmp_path):
    """With the library missing, the binding raises instead of computing."""
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        _lib.load()


def test_library_built_from_these_sources(lib):
    from paper_1211_4864_amd import build
    assert lib.hacc_sr_source_hash().decode() == build.source_hash()


def test_stale_library_is_refused(lib, monkeypatch):
    """A library whose embedded source hash differs from the sources in the
    tree is refused at load time."""
    from paper_1211_4864_amd import build
    monkeypatch.setattr(build, "source_hash", lambda: "0" * 64)
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(_lib.StaleLibraryError):
        _lib.load()


def test_rcb_and_pm_argument_validation(lib):
    poly = _poly()
    # leaf_max outside 1..2^20
    assert lib.hacc_sr_force_rcb(P(16), P(16), 10, 1.0, F(0.1), F(1e-5), poly, 0,
                                 P(16)) == -1
    assert lib.hacc_sr_force_vjp_rcb(P(16), P(16), 10, 1.0, F(0.1), F(1e-5), poly,
                                     (1 << 20) + 1, P(16), P(16)) == -1
    out = ctypes.c_size_t(0)
    assert lib.hacc_sr_workspace_bytes_rcb(1000, 1.0, F(0.1), ctypes.byref(out)) == 0
    base = ctypes.c_size_t(0)
    assert lib.hacc_sr_workspace_bytes(1000, 1.0, F(0.1), ctypes.byref(base)) == 0
    assert out.value > base.value
    # PM: power-of-two grid 8..512, periodic box, sigma >= 0, 0 <= n_s <= 16
    for ng in (4, 12, 1024):
        assert lib.hacc_sr_pm_accel(P(16), P(16), 10, 1.0, ng, F(0.8), 3, P(16)) == -1
    assert lib.hacc_sr_pm_accel(P(16), P(16), 10, -1.0, 64, F(0.8), 3, P(16)) == -1
    assert lib.hacc_sr_pm_accel(P(16), P(16), 10, 1.0, 64, F(-0.1), 3, P(16)) == -1
    assert lib.hacc_sr_pm_accel(P(16), P(16), 10, 1.0, 64, F(0.8), 17, P(16)) == -1
    assert lib.hacc_sr_pm_accel(None, None, 0, 1.0, 64, F(0.8), 3, None) == 0
    assert lib.hacc_sr_pm_workspace_bytes(256, 1000, ctypes.byref(out)) == 0
    assert out.value >= 2 * 8 * 256 ** 3 + 4 * 4 * 1000
    small = out.value
    assert lib.hacc_sr_pm_workspace_bytes(256, 10 ** 6, ctypes.byref(out)) == 0
    assert out.value > small
    assert lib.hacc_sr_pm_workspace_bytes(256, -1, ctypes.byref(out)) == -1
    assert lib.hacc_sr_pm_workspace_bytes(12, 10, ctypes.byref(out)) == -1


def test_binned_vjp_refuses_without_token(lib):
    """No GPU work: a token of 0 (or one never issued) is refused before any
    launch, and the token query validates its pointer."""
    P, F = ctypes.c_void_p, ctypes.c_float
    poly = (ctypes.c_float * 6)(*([0.0] * 6))
    tok = ctypes.c_uint64(7)
    assert lib.hacc_sr_binning_token(None) == -1
    assert lib.hacc_sr_binning_token(ctypes.byref(tok)) == 0
    assert tok.value == 0
    for t in (0, 12345):
        assert lib.hacc_sr_force_vjp_binned(ctypes.c_uint64(t), 100, 1.0, F(0.05), F(1e-4),
                                            poly, P(16), P(16)) == -5
    # argument checks come first; n = 0 is a no-op
    assert lib.hacc_sr_force_vjp_binned(ctypes.c_uint64(0), 100, 1.0, F(-0.05), F(1e-4),
                                        poly, P(16), P(16)) == -1
    assert lib.hacc_sr_force_vjp_binned(ctypes.c_uint64(0), 0, 1.0, F(0.05), F(1e-4),
                                        poly, None, None) == 0
    assert "token" in _lib.strerror(-5)
