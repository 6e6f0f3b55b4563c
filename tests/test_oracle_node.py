"""Pins of the oracle's tables and single-node operators against what the paper and the
mathematics fix (printed tables, isotropy identities, equilibrium moments, a numerical solve of
the central-moment transform, the Akai construction, conservation of the collision)."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_lattice_is_printed_matrix_M(oracle_mod):
    M = np.array(_read_rows("d3q19_matrix_M.txt"), dtype=int)
    c, w, opp = oracle_mod.lattice()
    assert np.array_equal(c.T, M)
    for i in range(19):
        assert np.array_equal(c[opp[i]], -c[i])


def test_weights_are_printed_tables(oracle_mod):
    rows = _read_rows("weights.txt")
    d3 = {int(r[1]): float(r[2]) / float(r[3]) for r in rows if r[0] == "d3q19"}
    e8w = {int(r[1]): float(r[2]) / float(r[3]) for r in rows if r[0] == "e8"}
    c, w, _ = oracle_mod.lattice()
    for i in range(19):
        assert w[i] == d3[int((c[i] ** 2).sum())]
    e, we = oracle_mod.e8()
    assert len(e) == 92
    assert len({tuple(v) for v in e}) == 92
    for v, om in zip(e, we):
        assert om == e8w[int((v ** 2).sum())]


def test_d3q19_isotropy(oracle_mod):
    c, w, _ = oracle_mod.lattice()
    c = c.astype(float)
    d = np.eye(3)
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(np.einsum("i,ia->a", w, c)).max() < 1e-16
    assert np.abs(np.einsum("i,ia,ib->ab", w, c, c) - d / 3).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, c, c, c)).max() < 1e-16
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.abs(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c) - iso4).max() < 1e-15


def test_e8_isotropy(oracle_mod):
    e, w = oracle_mod.e8()
    e = e.astype(float)
    assert np.abs(np.einsum("i,ia,ib->ab", w, e, e) - np.eye(3)).max() < 1e-14
    # fourth-order isotropy: sum w e_x^4 = 3 sum w e_x^2 e_y^2
    assert abs((w * e[:, 0] ** 4).sum() - 3 * (w * e[:, 0] ** 2 * e[:, 1] ** 2).sum()) < 1e-14


def test_equilibrium_moments(oracle_mod):
    rng = np.random.default_rng(0)
    c, _, _ = oracle_mod.lattice()
    c = c.astype(float)
    for _ in range(50):
        rho = rng.uniform(0.5, 1.5)
        u = rng.uniform(-0.1, 0.1, 3)
        f = oracle_mod.feq(rho, u)
        assert abs(f.sum() - rho) < 1e-14
        assert np.abs(f @ c - rho * u).max() < 1e-15
        assert np.abs(np.einsum("i,ia,ib->ab", f, c, c) - rho * (np.outer(u, u) + np.eye(3) / 3)).max() < 1e-14
        # the shear central moments k5..k9 of the equilibrium vanish
        cb = c - u
        k = [f @ (cb[:, 0] ** 2 - cb[:, 1] ** 2), f @ (cb[:, 1] ** 2 - cb[:, 2] ** 2),
             f @ (cb[:, 0] * cb[:, 1]), f @ (cb[:, 0] * cb[:, 2]), f @ (cb[:, 1] * cb[:, 2])]
        assert np.abs(k).max() < 1e-15


def transform_T(c, u):
    """T of Appendix A, built from the moment vectors t_i (eq. forward_transformation_vector)."""
    cb = c.astype(float) - u
    x, y, z = cb[:, 0], cb[:, 1], cb[:, 2]
    rows = [np.ones(19), x, y, z, x * x + y * y + z * z, x * x - y * y, y * y - z * z, x * y, x * z, y * z,
            x * x * y, x * y * y, x * x * z, x * z * z, y * y * z, y * z * z, x * x * y * y, x * x * z * z,
            y * y * z * z]
    return np.array(rows)


def test_cm_closed_form_inverts_T(oracle_mod):
    """The printed T^{-1} k* equals a numerical solve of T d = (0,..,k5..k9,..,0)."""
    rng = np.random.default_rng(1)
    c, _, _ = oracle_mod.lattice()
    for trial in range(200):
        u = rng.uniform(-0.3, 0.3, 3) if trial else np.zeros(3)
        k = rng.normal(size=5)
        d = oracle_mod.cm_back(u, k)
        T = transform_T(c, u)
        assert abs(np.linalg.det(T) + 98304) < 1e-7
        rhs = np.zeros(19)
        rhs[5:10] = k
        assert np.abs(T @ d - rhs).max() < 1e-13
        assert np.abs(d - np.linalg.solve(T, rhs)).max() < 1e-13


def test_cm_closed_form_each_column(oracle_mod):
    """Each of the five printed columns matches the corresponding column of T^{-1}."""
    rng = np.random.default_rng(2)
    c, _, _ = oracle_mod.lattice()
    for _ in range(20):
        u = rng.uniform(-0.2, 0.2, 3)
        Tinv = np.linalg.inv(transform_T(c, u))
        for j in range(5):
            k = np.zeros(5)
            k[j] = 1.0
            assert np.abs(oracle_mod.cm_back(u, k) - Tinv[:, 5 + j]).max() < 1e-13


def test_akai_realignment(oracle_mod):
    """n*.n_s = cos(theta), |n*| = 1, and the nearest candidate is always n+."""
    rng = np.random.default_rng(3)
    for _ in range(2000):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        ns = rng.normal(size=3)
        ns /= np.linalg.norm(ns)
        th = rng.uniform(0.01, np.pi - 0.01)
        out, npl, nmi = oracle_mod.wetting(n, ns, th)
        assert abs(np.linalg.norm(npl) - 1) < 1e-12 and abs(np.linalg.norm(nmi) - 1) < 1e-12
        assert abs(npl @ ns - np.cos(th)) < 1e-12
        assert abs(nmi @ ns - np.cos(th)) < 1e-12
        # n+ lies in the plane of n and n_s, on the same side of n_s as n, and is the nearer one
        assert abs(np.cross(n, ns) @ npl) < 1e-12
        assert np.linalg.norm(npl - n) <= np.linalg.norm(nmi - n)
        if np.linalg.norm(np.cross(n, ns)) >= 1e-2:
            assert np.array_equal(out, npl)


def test_akai_cone_keeps_normal(oracle_mod):
    """Within 1e-2 rad of +-n_s (no rotation plane) n is kept; just outside, n+ is used."""
    ns = np.array([0.0, 0.0, 1.0])
    th = np.deg2rad(60)
    for sign in (1.0, -1.0):
        for e in (0.0, 1e-12, 1e-6, 9.9e-3, 1.01e-2, 0.1):
            n = np.array([e, 0.0, sign])
            n /= np.linalg.norm(n)
            out, npl, _ = oracle_mod.wetting(n, ns, th)
            if np.linalg.norm(np.cross(n, ns)) < 1e-2:
                assert np.array_equal(out, n)
            else:
                assert np.array_equal(out, npl)
                assert abs(out @ ns - np.cos(th)) < 1e-12


def _one_node(oracle_mod, fr, fp, **kw):
    o = oracle_mod.Oracle((1, 1, 1), rho_r0=1.0, rho_p0=0.0, **kw)
    o.set_state(fr.reshape(19, 1), fp.reshape(19, 1), np.full((7, 1), 1 / 7.0))
    return o


def test_tau_one_is_bgk_with_shifted_velocity(oracle_mod):
    """At tau = 1 the collision returns sum_k f^eq(rho^k, u + du^k), split by colour share."""
    rng = np.random.default_rng(4)
    c, w, _ = oracle_mod.lattice()
    fr = w * rng.uniform(0.3, 0.9) * (1 + 0.2 * rng.uniform(-1, 1, 19))
    fp = w * rng.uniform(0.1, 0.5) * (1 + 0.2 * rng.uniform(-1, 1, 19))
    a = np.array([[1e-3, -2e-3, 5e-4], [-1e-3, 3e-3, 2e-4]])
    o = _one_node(oracle_mod, fr, fp, tau=1.0, accel=a)
    o.step(1)
    sr, sp, _ = o.get_state()
    rr, rp = fr.sum(), fp.sum()
    rm = rr + rp
    u = (fr + fp) @ c / rm
    fstar = oracle_mod.feq(rr, u + a[0]) + oracle_mod.feq(rp, u + a[1])
    assert np.abs(sr[:, 0] - rr / rm * fstar).max() < 1e-15
    assert np.abs(sp[:, 0] - rp / rm * fstar).max() < 1e-15


def test_collision_conserves_mass_and_adds_impulse(oracle_mod):
    rng = np.random.default_rng(5)
    c, w, _ = oracle_mod.lattice()
    for tau in (0.55, 0.8, 1.7):
        fr = w * (0.7 + 0.3 * rng.uniform(-1, 1, 19))
        fp = w * (0.3 + 0.2 * rng.uniform(-1, 1, 19))
        a = rng.uniform(-1e-3, 1e-3, (2, 3))
        o = _one_node(oracle_mod, fr, fp, tau=tau, accel=a)
        o.step(1)
        sr, sp, _ = o.get_state()
        assert abs(sr.sum() - fr.sum()) < 1e-15 and abs(sp.sum() - fp.sum()) < 1e-15
        mom = (sr[:, 0] + sp[:, 0]) @ c
        expect = (fr + fp) @ c + fr.sum() * a[0] + fp.sum() * a[1]
        assert np.abs(mom - expect).max() < 1e-15
        # the relaxed shear central moments about the bare velocity scale by (1 - 1/tau) when
        # there is no force
        o = _one_node(oracle_mod, fr, fp, tau=tau)
        o.step(1)
        sr, sp, _ = o.get_state()
        fm, fs = fr + fp, sr[:, 0] + sp[:, 0]
        u = fm @ c / fm.sum()
        cb = c - u
        def shear(f):
            return np.array([f @ (cb[:, 0] ** 2 - cb[:, 1] ** 2), f @ (cb[:, 1] ** 2 - cb[:, 2] ** 2),
                             f @ (cb[:, 0] * cb[:, 1]), f @ (cb[:, 0] * cb[:, 2]), f @ (cb[:, 1] * cb[:, 2])])
        assert np.abs(shear(fs) - (1 - 1 / tau) * shear(fm)).max() < 1e-15
