"""The C-ABI library loads without a GPU, exports every symbol the header declares, and rejects
invalid arguments on the host before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def core():
    from paper_2608_15781_amd import build, core as c

    if build.stale():
        build.build()
    return c


def test_exports_every_declared_symbol(core):
    header = open(os.path.join(ROOT, "include", "lbm.h")).read()
    header = re.sub(r"/\*.*?\*/", "", header, flags=re.S)
    declared = set(re.findall(r"\b(lbm_[a-z_]+)\(", header))
    assert declared, "no declarations found"
    L = core.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert set(core.EXPORTED) == declared


def test_version(core):
    assert b"gfx950" in core.lib().lbm_version()


def test_workspace_sizes_scale_with_precision(core):
    sizes = {}
    for prec in ("fp64", "fp32", "fp16", "bf16"):
        p = core.make_params((64, 64, 64), precision=prec, tau=0.8, species=True)
        b = ctypes.c_size_t()
        assert core.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(b)) == 0
        s = ctypes.c_size_t()
        assert core.lib().lbm_state_bytes(ctypes.byref(p), ctypes.byref(s)) == 0
        sizes[prec] = (b.value, s.value)
    N = 64 ** 3
    # state = 19 populations + 4 scalars + 7 species populations per node (+ the species total in
    # the arithmetic type with 2-byte storage)
    assert sizes["fp64"][1] >= (19 + 4 + 7) * 8 * N
    assert sizes["fp32"][1] >= (19 + 4 + 7) * 4 * N
    assert sizes["fp16"][1] >= (19 + 7) * 2 * N + (4 + 1) * 4 * N
    assert sizes["fp16"][1] < sizes["fp32"][1] < sizes["fp64"][1]


@pytest.mark.parametrize("species", [True, False])
@pytest.mark.parametrize("prec,s,r", [("fp64", 8, 8), ("fp32", 4, 4), ("fp16", 2, 4), ("bf16", 2, 4)])
def test_state_layout_and_plane_stride(core, prec, s, r, species):
    """The population planes, colour scalars and species planes fit in the reported state size, and
    planes are an odd multiple of 256 bytes apart (equal entries of different planes do not share
    a memory channel when N is a power of two)."""
    N = 64 ** 3
    p = core.make_params((64, 64, 64), precision=prec, tau=0.8, species=species)
    f, a, g, ps = (ctypes.c_size_t() for _ in range(4))
    assert core.lib().lbm_state_layout(ctypes.byref(p), ctypes.byref(f), ctypes.byref(a), ctypes.byref(g),
                                       ctypes.byref(ps)) == 0
    assert ps.value >= N and (ps.value * s) % 256 == 0 and (ps.value * s // 256) % 2 == 1
    assert f.value == 0 and a.value >= 19 * s * ps.value and g.value >= a.value + 4 * r * ps.value
    sb = ctypes.c_size_t()
    assert core.lib().lbm_state_bytes(ctypes.byref(p), ctypes.byref(sb)) == 0
    cplane = r * ps.value if (species and s == 2) else 0  # species totals after the 2-byte planes
    assert sb.value >= g.value + (7 * s * ps.value if species else 0) + cplane
    ab, scr = ctypes.c_size_t(), ctypes.c_size_t()
    assert core.lib().lbm_adjoint_bytes(ctypes.byref(p), ctypes.byref(ab), ctypes.byref(scr)) == 0
    assert ab.value >= 30 * r * ps.value


@pytest.mark.parametrize("field,value", [("tau", 0.5), ("tau", float("nan")), ("sigma", -1.0), ("beta", -0.1),
                                         ("xi", -1e-3), ("grad_eps", 0.0), ("nx", 0), ("precision", 7),
                                         ("fluid_nodes", -1), ("fluid_nodes", 8 ** 3 + 1),
                                         ("fp16_scale_log2", 40)])
def test_invalid_params_rejected(core, field, value):
    p = core.make_params((8, 8, 8), precision="fp16", tau=0.8)
    setattr(p, field, value)
    b = ctypes.c_size_t()
    assert core.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(b)) == core.LBM_ERR_ARG
    assert core.lib().lbm_last_error(None)


@pytest.mark.parametrize("prec,s,r", [("fp64", 8, 8), ("fp32", 4, 4), ("fp16", 2, 4), ("bf16", 2, 4)])
def test_layout_sized_by_fluid_nodes(core, prec, s, r):
    """With the mask's fluid count the planes hold that many entries (not one per node): the
    state, adjoint and fields buffers shrink with the porosity, and the workspace still has room
    for the 34 bytes per node that lbm_init stages."""
    shape = (64, 48, 40)
    N = 64 * 48 * 40

    def sizes(nf):
        p = core.make_params(shape, precision=prec, tau=0.8, species=True, fluid_nodes=nf)
        out = [ctypes.c_size_t() for _ in range(6)]
        assert core.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(out[0])) == 0
        assert core.lib().lbm_state_bytes(ctypes.byref(p), ctypes.byref(out[1])) == 0
        assert core.lib().lbm_adjoint_bytes(ctypes.byref(p), ctypes.byref(out[2]), ctypes.byref(out[3])) == 0
        assert core.lib().lbm_fields_bytes(ctypes.byref(p), ctypes.byref(out[4])) == 0
        f, a, g = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        assert core.lib().lbm_state_layout(ctypes.byref(p), ctypes.byref(f), ctypes.byref(a), ctypes.byref(g),
                                           ctypes.byref(out[5])) == 0
        return [o.value for o in out]

    ws_all, sb_all, ab_all, _, fb_all, ps_all = sizes(0)
    nf = N // 2 + 37
    ws, sb, ab, scr, fb, ps = sizes(nf)
    unit = 256 // s
    assert nf <= ps < nf + 2 * unit and ps_all >= N
    assert sb >= (26 * s + 4 * r) * ps and sb < 0.55 * sb_all
    assert ab >= 30 * r * ps and ab < 0.55 * ab_all
    assert fb < fb_all and ws < ws_all
    assert ws >= 2 * sb
    # a nearly solid lattice: the init staging, not the state, sets the size of the tail
    ws1 = sizes(1)[0]
    assert ws1 >= 34 * N


def test_largest_lattice_sizes(core):
    """nx*ny*nz just below 2^31 is accepted and its sizes do not overflow; one plane more is refused."""
    shape = (1290, 1290, 1290)  # 2,146,689,000 nodes
    N = 1290 ** 3
    for prec, s, r in (("fp64", 8, 8), ("fp32", 4, 4), ("fp16", 2, 4)):
        for nf in (0, N // 2):
            p = core.make_params(shape, precision=prec, tau=0.8, species=True, fluid_nodes=nf)
            ws, sb = ctypes.c_size_t(), ctypes.c_size_t()
            assert core.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(ws)) == 0
            assert core.lib().lbm_state_bytes(ctypes.byref(p), ctypes.byref(sb)) == 0
            F = nf or N
            assert sb.value >= (26 * s + 4 * r) * F
            assert ws.value >= 2 * sb.value + 4 * N * 3
    p = core.make_params((1291, 1290, 1290), precision="fp32", tau=0.8)
    b = ctypes.c_size_t()
    assert core.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(b)) == core.LBM_ERR_ARG
    assert b"2^31" in core.lib().lbm_last_error(None)


def test_open_species_planes_need_two_x_layers(core):
    """With the species inlet and outflow planes on, nx = 1 would make them one plane: refused."""
    b = ctypes.c_size_t()
    p = core.make_params((1, 8, 8), precision="fp32", tau=0.8, species=True, x_open=True)
    assert core.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(b)) == core.LBM_ERR_ARG
    assert b"x_open" in core.lib().lbm_last_error(None)
    for shape, kw in (((2, 8, 8), dict(species=True, x_open=True)), ((1, 8, 8), dict(species=True)),
                      ((1, 8, 8), dict(x_open=True))):
        p = core.make_params(shape, precision="fp32", tau=0.8, **kw)
        assert core.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(b)) == 0


def _init(core, p, N, ws_bytes, rho_r0=None, theta=None, ws_ptr=256):
    solid = np.zeros(N, np.uint8)
    rr = np.ones(N) if rho_r0 is None else rho_r0
    rp = np.zeros(N)
    h = ctypes.c_void_p()
    P = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    return core.lib().lbm_init(ctypes.byref(p), P(solid), P(theta), 1.0, None, P(rr), P(rp), None,
                               ctypes.c_void_p(ws_ptr), ws_bytes, None, ctypes.byref(h))


def test_init_rejects_bad_inputs_on_host(core):
    """Checked before any device call: small or misaligned workspace, bad densities or angles."""
    p = core.make_params((4, 4, 4), precision="fp32", tau=0.8)
    N = 64
    need = ctypes.c_size_t()
    core.lib().lbm_workspace_bytes(ctypes.byref(p), ctypes.byref(need))
    assert _init(core, p, N, need.value - 1) == core.LBM_ERR_ARG
    assert b"too small" in core.lib().lbm_last_error(None)
    assert _init(core, p, N, need.value, ws_ptr=257) == core.LBM_ERR_ARG
    bad = np.ones(N)
    bad[5] = np.nan
    assert _init(core, p, N, need.value, rho_r0=bad) == core.LBM_ERR_ARG
    th = np.full(N, 4.0)
    assert _init(core, p, N, need.value, theta=th) == core.LBM_ERR_ARG
    assert b"theta" in core.lib().lbm_last_error(None)
    # a fluid count that does not match the mask (all 64 nodes are fluid)
    p.fluid_nodes = 63
    assert _init(core, p, N, need.value) == core.LBM_ERR_ARG
    assert b"fluid_nodes" in core.lib().lbm_last_error(None)


def test_binding_fails_loudly_without_library(monkeypatch, core):
    from paper_2608_15781_amd import build

    monkeypatch.setattr(core, "_lib", None)
    monkeypatch.setattr(build, "LIB", "/nonexistent/liblbm.so")
    with pytest.raises(RuntimeError, match="not built"):
        core.lib()
