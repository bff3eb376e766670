"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and validates parameters (no GPU compute calls)."""
import ctypes
import os
import re

import pytest

from paper_2311_10827_amd import _lib, inputs
from paper_2311_10827_amd.sim import make_params

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lbmwb.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(_lib.SYMBOLS)


def declared_struct_fields(name):
    """Field names of `typedef struct name {...}` in the header, in order."""
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct %s \{(.*?)\}" % name, txt, flags=re.S).group(1)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        names = decl.split(None, 1)[1]
        out += [re.sub(r"\[.*\]", "", v).strip() for v in names.split(",")]
    return out


@pytest.mark.parametrize("c_name,py_struct", [("lbm_params", _lib.LbmParams),
                                               ("lbm_derived", _lib.LbmDerived),
                                               ("lbm_diag", _lib.LbmDiag)])
def test_structs_mirror_the_header(c_name, py_struct):
    assert declared_struct_fields(c_name) == [f for f, _ in py_struct._fields_]


def test_library_exports_every_symbol():
    L = _lib.load()
    for name in declared_functions():
        assert hasattr(L, name), name


def _derive(p):
    d = _lib.LbmDerived()
    return _lib.load().lbm_derive(ctypes.byref(p), ctypes.byref(d)), d


def test_derive_from_sigma_W():
    rc, d = _derive(make_params(inputs.FLAT))
    assert rc == 0
    # Sec. 2.1, eqs. beta and suiface_tension, with sigma = 0.01, W = 4, dphi = 2
    assert d.kappa == pytest.approx(0.015, rel=1e-15)
    assert d.beta == pytest.approx(1.875e-3, rel=1e-15)
    assert d.sigma == pytest.approx(0.01, rel=1e-14)
    assert d.W == pytest.approx(4.0, rel=1e-14)
    # Sec. 2.3.1 eq. mobility and Sec. 2.3.2: tau = 1/2 + 3 M / alpha, 1/2 + 3 nu
    assert d.tau_f == pytest.approx(0.8, rel=1e-15)
    assert d.tau_gA == pytest.approx(0.8, rel=1e-15) and d.tau_gB == pytest.approx(0.8, rel=1e-15)
    rc, d = _derive(make_params(inputs.DROPLET))
    assert rc == 0 and d.tau_gA == pytest.approx(0.53) and d.tau_gB == pytest.approx(0.8)
    assert d.tau_f == pytest.approx(0.65)


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-3), dict(bc_x=2), dict(precision=16), dict(phi_A=-1.0),
    dict(rho_B=0.0), dict(rho_A=-2.0), dict(nu_A=0.0), dict(M=0.0), dict(alpha=0.0),
    dict(kappa=-1.0, beta=0.0), dict(diag_every=-1), dict(nx=65536, ny=65536),
    dict(gx=float("nan")), dict(kernel_path=3), dict(kernel_path=4), dict(kernel_path=-1),
    dict(kernel_path=3, precision=32, bc_x=1, bc_y=0), dict(kernel_path=3, precision=32, bc_x=0, bc_y=1),
    dict(nu_form=3),
    dict(nu_form=-1), dict(collision=2), dict(collision=1, mrt_f=(0.0, 1.0, 1.0, 1.0)),
    dict(collision=1, mrt_g=(1.0, 2.0)), dict(collision=1, mrt_f=(1.0, 1.0, float("nan"), 1.0)),
    dict(lo_format=3), dict(lo_format=-1), dict(use_tau=2),
])
def test_derive_rejects(bad):
    p = make_params(inputs.FLAT, **bad)
    rc, _ = _derive(p)
    assert rc == _lib.LBM_EINVAL
    assert _lib.load().lbm_state_bytes(ctypes.byref(p)) == 0


def test_two_step_path_is_for_fp32_on_periodic_grids():
    # kernel_path 3 (two steps per launch) takes FP32 with both directions
    # periodic; FP64 and walls are rejected above
    p = make_params(inputs.FLAT, precision=32, kernel_path=3, bc_x=0, bc_y=0)
    rc, d = _derive(p)
    assert rc == 0 and d.two_step == 1


@pytest.mark.parametrize("over,want", [
    (dict(precision=32, nx=4096, ny=4096), 1),          # state beyond the last-level cache
    (dict(precision=32, nx=1024, ny=1024), 0),          # 168 MiB: fits it
    (dict(precision=64, nx=4096, ny=4096), 0),
    (dict(precision=32, nx=4096, ny=4096, bc_x=1), 0),
    (dict(precision=32, nx=4096, ny=4096, kernel_path=2), 0),
    (dict(precision=32, nx=1024, ny=1024, kernel_path=3), 1),
])
def test_automatic_two_step_choice(over, want):
    rc, d = _derive(make_params(inputs.COALESCENCE, **over))
    assert rc == 0 and d.two_step == want


def test_derive_from_relaxation_times():
    # use_tau: alpha from eq. mobility solved for alpha, nu from the viscosity
    # relation of Sec. 2.3.2; the alpha and nu fields are ignored
    p = make_params(inputs.DROPLET, use_tau=1, tau_f=0.8, tau_gA=0.53, tau_gB=1.1, alpha=-5.0,
                    nu_A=-1.0, nu_B=0.0)
    rc, d = _derive(p)
    assert rc == 0
    assert (d.tau_f, d.tau_gA, d.tau_gB) == (0.8, 0.53, 1.1)
    assert d.alpha == pytest.approx(p.M / ((1 / 3) * 0.3), rel=1e-15)
    assert d.nu_A == pytest.approx(0.03 / 3, rel=1e-13) and d.nu_B == pytest.approx(0.6 / 3, rel=1e-15)
    # the same step from (M, alpha, nu) gives the same relaxation times
    q = make_params(inputs.DROPLET, alpha=d.alpha, nu_A=d.nu_A, nu_B=d.nu_B)
    rc, e = _derive(q)
    assert rc == 0
    for k in ("tau_f", "tau_gA", "tau_gB"):
        assert getattr(e, k) == pytest.approx(getattr(d, k), rel=1e-15)


@pytest.mark.parametrize("bad", [dict(tau_f=0.5), dict(tau_gA=0.4), dict(tau_gB=float("inf")),
                                 dict(tau_f=float("nan"))])
def test_derive_rejects_relaxation_times(bad):
    kw = dict(use_tau=1, tau_f=0.8, tau_gA=0.8, tau_gB=0.8)
    kw.update(bad)
    assert _derive(make_params(inputs.DROPLET, **kw))[0] == _lib.LBM_EINVAL


@pytest.mark.parametrize("prec,fmt,n,path,want", [
    (32, _lib.LO_AUTO, 512, 0, 0), (32, _lib.LO_AUTO, 8192, 2, 1), (32, _lib.LO_AUTO, 8192, 0, 0),
    (32, _lib.LO_AUTO, 8192, 3, 0), (32, _lib.LO_16, 512, 0, 1), (32, _lib.LO_16, 8192, 0, 1),
    (32, _lib.LO_32, 8192, 2, 0), (64, _lib.LO_16, 512, 0, 0)])
def test_low_word_format(prec, fmt, n, path, want):
    # automatic: 16 bits above a 1 GiB state (512^2 FP32 is 41 MiB, 8192^2 10 GiB)
    # for the one-step kernels; two steps per launch (automatic here on the
    # periodic 8192^2 grid) keep the 32-bit word
    rc, d = _derive(make_params(inputs.THROUGHPUT, precision=prec, nx=n, ny=n, lo_format=fmt,
                                kernel_path=path))
    assert rc == 0 and d.lo16 == want


def test_sigma_W_must_be_positive():
    p = make_params(inputs.FLAT)
    p.sigma = 0.0
    assert _derive(p)[0] == _lib.LBM_EINVAL


@pytest.mark.parametrize("prec,esz", [(64, 8), (32, 4)])
def test_state_bytes(prec, esz):
    p = make_params(inputs.FLAT, precision=prec)
    nb = _lib.load().lbm_state_bytes(ctypes.byref(p))
    # two population buffers (18 planes in FP64, 19 in FP32: f_0 as hi + lo),
    # plus two S planes, phi, mu, each plane at least nx*ny cells
    planes = 40 if prec == 64 else 42
    assert nb >= planes * 256 * 4 * esz and nb % 256 == 0
    big = make_params(inputs.THROUGHPUT, precision=prec)
    nbb = _lib.load().lbm_state_bytes(ctypes.byref(big))
    assert planes * 16384 * 16384 * esz <= nbb < planes * 16384 * 16384 * esz * 1.001


def test_init_rejects_null_and_misaligned():
    L = _lib.load()
    p = make_params(inputs.FLAT)
    ctx = ctypes.c_void_p()
    assert L.lbm_init(ctypes.byref(ctx), ctypes.byref(p), None, None, None, None, None, None) == _lib.LBM_EINVAL
    assert L.lbm_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.c_void_p(0x1001),
                      ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000), None, None, None) == _lib.LBM_EINVAL
    assert L.lbm_init(None, ctypes.byref(p), None, None, None, None, None, None) == _lib.LBM_EINVAL


def test_strerror_and_null_context():
    L = _lib.load()
    for code in (0, -1, -2, -3, -4, 7):
        assert isinstance(L.lbm_strerror(code), bytes)
    assert L.lbm_step(None, 1) == _lib.LBM_EINVAL
    assert L.lbm_step_count(None) == -1
    assert L.lbm_destroy(None) == 0
    assert L.lbm_stream_copy(None, None, 16, None) == _lib.LBM_EINVAL
    buf = (ctypes.c_double * 6)()
    assert L.lbm_adjoint_theta(None, _lib.THETA_TAU, buf, 0) == _lib.LBM_EINVAL
