"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function the public headers declare, and validates arguments before any launch."""

import ctypes
import json
import os
import re

import numpy as np
import pytest

from paper_1910_10908_amd import _lib, scenes
from paper_1910_10908_amd import tffr as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = []
    for h in ("tffr.h", "tffr_debug.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(tffr_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    lib = _lib.load()
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib._PROTOS), set(names) ^ set(_lib._PROTOS)


def test_params_struct_matches_header_order():
    text = open(os.path.join(ROOT, "include", "tffr.h")).read()
    body = text[text.index("typedef struct {"):text.index("} tffr_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"(int32_t|double)\s+([a-z0-9_, ]+);", body)
    flat = []
    for ty, names in fields:
        for n in names.split(","):
            flat.append((n.strip(), ty))
    assert [f[0] for f in _lib.Params._fields_] == [f[0] for f in flat]
    for (n, ct), (n2, ty) in zip(_lib.Params._fields_, flat):
        assert (ct is ctypes.c_double) == (ty == "double"), n


def test_defaults_are_the_paper_constants():
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_constants.json")))
    p = T.default_params()
    assert p.window_a == gold["window_a"]
    assert p.tau == gold["tffr_tau"]
    assert p.band_r == gold["ffr_band_r"]
    assert p.weighting == T.W_TFFR and p.thresh_mode == T.THRESH_LITERAL


def _ok_params(**kw):
    base = dict(n_pulses=8, n_freq=16, mx=16, my=16, fov_x=40.0, fov_y=40.0)
    base.update(kw)
    return T.default_params(**base)


def test_validate_accepts_paper_geometry():
    for wl in scenes.WORKLOADS.values():
        k, ku = scenes.radar_sampling(wl.n_pulses, wl.n_freq)
        p = _ok_params(n_pulses=wl.n_pulses, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov)
        assert T.tffr_validate(p, k, ku) == 0, wl.name


@pytest.mark.parametrize("name,kw,code", [
    ("ffr_vs_tffr_c64", {}, 0),                # full rank: selected inversion of the product
    ("precision_2k", {}, 0),                   # rank deficient, spacing 0.39-0.46: Gram route
    ("full_swath_4k", {}, 0),                  # rank deficient, spacing 0.20-0.23
    ("autofocus_1k", {}, 0),                   # routed; its numerical singularity shows at plan time
    ("precision_2k", dict(q=3.5), 5),          # Gram route needs q <= 3
    ("ffr_vs_tffr_c64", dict(q=4.5), 5),       # more than 11 lattice taps per sample
    ("ffr_vs_tffr_c64", dict(band_r=8), 0),    # band 8 still within the direct route
])
def test_validate_ffr_routes(name, kw, code):
    """Host-side route choice of plain FFR: which geometries the plan can solve."""
    wl = scenes.WORKLOADS[name]
    k, ku = scenes.radar_sampling(wl.n_pulses, wl.n_freq)
    p = _ok_params(n_pulses=wl.n_pulses, n_freq=wl.n_freq, mx=wl.m, my=wl.m, fov_x=wl.fov, fov_y=wl.fov,
                   weighting=T.W_FFR, **kw)
    assert T.tffr_validate(p, k, ku) == code


@pytest.mark.parametrize("kw,code", [
    (dict(n_pulses=0), 1), (dict(n_freq=0), 1), (dict(mx=15), 1), (dict(my=0), 1),
    (dict(fov_x=0.0), 1), (dict(fov_y=-1.0), 1), (dict(weighting=7), 1), (dict(window_a=-0.1), 1),
    (dict(q=0.5), 1), (dict(band_r=9), 1), (dict(tau=0.0), 1), (dict(thresh_mode=2), 1),
    (dict(kernel_width=1), 5), (dict(kernel_width=17), 5), (dict(upsampfac=1.0), 5), (dict(dtype=9), 5),
    (dict(mx=32768), 5),
])
def test_validate_rejects_bad_params(kw, code):
    k, ku = scenes.radar_sampling(8, 16)
    assert T.tffr_validate(_ok_params(**kw), k, ku) == code


def test_validate_geometry_errors():
    k, ku = scenes.radar_sampling(8, 16)
    p = _ok_params()
    bad = ku.copy()
    bad[3] = 2.0 * k[0]  # 4 k^2 - ku^2 = 0: evanescent
    assert T.tffr_validate(p, k, bad) == 2
    kk = k.copy()
    kk[5] = kk[4]
    assert T.tffr_validate(p, kk, ku) == 3
    kk = k.copy()
    kk[2] = np.nan
    assert T.tffr_validate(p, kk, ku) == 1


def test_validate_xy_layout_and_order():
    """Explicit coordinates: ky must be one value along each slice (TFFR_ERR_LAYOUT),
    kx strictly increasing along it (TFFR_ERR_NONMONOTONE), values finite (TFFR_ERR_ARG)."""
    k, ku = scenes.radar_sampling(8, 16)
    p = _ok_params()
    kx = np.sqrt(4 * k[None, :] ** 2 - ku[:, None] ** 2)
    ky = np.repeat(ku[:, None], 16, axis=1)
    assert T.tffr_validate_xy(p, kx, ky) == 0
    bad = ky.copy()
    bad[2, 7] += 1e-9
    assert T.tffr_validate_xy(p, kx, bad) == 4
    bad = kx.copy()
    bad[5, 9] = bad[5, 8]
    assert T.tffr_validate_xy(p, bad, ky) == 3
    bad = kx.copy()
    bad[1, 1] = np.inf
    assert T.tffr_validate_xy(p, bad, ky) == 1
    # non-Stolt geometry with the slice structure is accepted
    rng = np.random.default_rng(0)
    jit = kx + rng.uniform(-0.1, 0.1, kx.shape) * np.diff(kx, axis=1).min()
    assert T.tffr_validate_xy(p, jit, ky) == 0


def test_status_strings():
    lib = _lib.load()
    for code, name in _lib.STATUS_NAMES.items():
        assert lib.tffr_status_string(code).decode().startswith(name)


def test_null_handles_are_rejected_without_device():
    lib = _lib.load()
    assert lib.tffr_workspace_bytes(None) == 0
    assert lib.tffr_forward(None, None, None, None, None, None, None, None) == 1
    assert lib.tffr_adjoint(None, None, None, None, None, None, None, None, None, None, None) == 1
    assert lib.tffr_entropy(None, None, None, None, None, None) == 1
    assert lib.tffr_weights(None, None, None, None) == 1
    assert lib.tffr_row_phase_grad(None, None, None, None, None, None) == 1
    assert lib.tffr_coord_grad(None, None, None, None, None, None, None, None, None, None) == 1
    assert lib.tffr_debug_plan_config(None, None, None, None) == 1
    assert lib.tffr_rma_front_end_pos(None, None, 64, 1.0, None, 0.0, None, None) == 1
    assert lib.tffr_rma_range_fft(None, None, 1, None, None, None) == 1
    assert lib.tffr_debug_ent_cols(None, None, None, None, None, None) == 1
    assert lib.tffr_debug_ent_adj_rows(*([None] * 11)) == 1
    assert lib.tffr_debug_step_kernel_times(*([None] * 12), 10, None, None, None) == 1
    assert lib.tffr_debug_step_kernel_marginal_times(*([None] * 12), 10, None, None, None) == 1
    assert lib.tffr_debug_fft(3, 1, 1, 8, 0, None, None, None) == 1
    out = ctypes.c_void_p()
    k, ku = scenes.radar_sampling(8, 16)
    bad = _ok_params(n_pulses=0)
    assert lib.tffr_plan_create(ctypes.byref(bad), k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                ku.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(out)) == 1
    assert not out.value
    kx = np.ones((8, 16))
    assert lib.tffr_plan_create_xy(ctypes.byref(bad), kx.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   kx.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(out)) == 1
    assert not out.value
