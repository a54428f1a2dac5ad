"""CPU checks of the library's point physics (host build of the same header
the kernels use): forward fluxes against the oracle's, and every hand-written
vector-Jacobian product against central differences of the forward code,
<w, J d> = <J^T w, d>, on both branches of the log mean and of Rusanov's
wave-speed maximum."""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
G = 1.4
C = np.array([G, 0.02, 0.72, 1.0, 0.0, 0.0, 0.0, 1.0, 0.4])    # gamma, mu, Pr, R, riemann, twopoint, visc law, Tref, Ts
_dp = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def pw():
    path = os.path.join(ROOT, "paper_2605_28627_amd", "libdgx_pointwise_check.so")
    if not os.path.exists(path):
        from paper_2605_28627_amd import build
        build.build_pointwise_check()
    return ctypes.CDLL(path)


def P(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.ctypes.data_as(_dp)


def state(rng, scale=1.0, base=None):
    if base is not None:
        return base * (1 + scale * rng.uniform(-1, 1, 5))
    rho = rng.uniform(0.6, 1.6)
    u = rng.uniform(-0.8, 0.8, 3)
    p = rng.uniform(0.6, 1.6)
    return np.array([rho, *(rho * u), p / (G - 1) + 0.5 * rho * u @ u])


def call(f, nout, *args):
    out = np.zeros(nout)
    f(*[P(a) if isinstance(a, np.ndarray) else a for a in args], P(out))
    return out


def fd_dot(fwd, x, d, w, eps=1e-6):
    return w @ ((fwd(x + eps * d) - fwd(x - eps * d)) / (2 * eps))


def test_forward_matches_oracle(pw, orc):
    rng = np.random.default_rng(0)
    for _ in range(30):
        a, b = state(rng), state(rng)
        n = rng.normal(size=3)
        F = call(pw.pw_chandrashekar, 5, a, b, n, C)
        assert np.allclose(F, orc.flux_twopoint(a, b, n), rtol=1e-13, atol=1e-13)
        F = call(pw.pw_euler_flux, 5, a, n, C)
        assert np.allclose(F, orc.flux_adv(a, n), rtol=1e-13, atol=1e-13)
        g = rng.normal(size=12)
        Gn = call(pw.pw_viscous_flux, 4, a, g, n, C)
        ref = sum(n[d] * orc.flux_visc(a, g, d, mu=C[1], Pr=C[2]) for d in range(3))
        assert np.allclose(Gn, ref[1:], rtol=1e-13, atol=1e-13)
    # float two-point flux: float-level agreement
    a, b = state(rng), state(rng)
    n = rng.normal(size=3)
    F32 = call(pw.pw_chandrashekar_f32, 5, a, b, n, C)
    assert np.allclose(F32, orc.flux_twopoint(a, b, n), rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("form", [0, 1])
def test_roe_surface_flux_matches_oracle(pw, orc, form):
    """The library's Roe flux (Harten-Hyman fix) against the oracle's, on random
    pairs and on pairs straddling a sonic point (where the fix acts)."""
    rng = np.random.default_rng(21 + form)
    c = C.copy()
    c[4] = 2
    g0 = np.zeros(12)
    for it in range(40):
        nh = rng.normal(size=3)
        nh /= np.linalg.norm(nh)
        if it % 2:
            a, b = state(rng), state(rng)
        else:                                   # un - c changes sign between the sides
            cs = np.sqrt(G)
            a = np.array([1.0, *((cs - 0.05) * nh), 1 / 0.4 + 0.5 * (cs - 0.05) ** 2])
            b = np.array([1.0, *((cs + 0.05) * nh), 1 / 0.4 + 0.5 * (cs + 0.05) ** 2])
        s = rng.uniform(0.5, 2.0)
        out = np.zeros(5)
        pw.pw_surface_flux(form, 0, P(a), P(b), P(g0), P(g0), P(nh), ctypes.c_double(s), P(c), P(out))
        central = orc.flux_twopoint(a, b, nh * s) if form else 0.5 * (orc.flux_adv(a, nh * s) + orc.flux_adv(b, nh * s))
        ref = central - 0.5 * s * orc.roe_matrix(a, b, nh, 0)
        assert np.allclose(out, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max()), (out, ref)


def test_sutherland_viscous_flux_matches_oracle(pw, orc):
    rng = np.random.default_rng(23)
    c = C.copy()
    c[6], c[7], c[8] = 1.0, 0.7, 0.4
    for _ in range(30):
        a = state(rng)
        n = rng.normal(size=3)
        g = rng.normal(size=12)
        Gn = call(pw.pw_viscous_flux, 4, a, g, n, c)
        ref = sum(n[d] * orc.flux_visc_law(a, g, d, mu=c[1], Pr=c[2], law=1, Tref=0.7, Ts=0.4) for d in range(3))
        assert np.allclose(Gn, ref[1:], rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("near", [False, True], ids=["direct-branch", "series-branch"])
def test_chandrashekar_vjp(pw, near):
    rng = np.random.default_rng(1)
    for _ in range(40):
        a = state(rng)
        b = state(rng, 1e-4, a) if near else state(rng)
        n = rng.normal(size=3)
        w = rng.normal(size=5)
        d = rng.normal(size=5) * np.abs(a)
        vjp = call(pw.pw_chandrashekar_vjp_a, 5, a, b, n, C, w)
        ref = fd_dot(lambda x: call(pw.pw_chandrashekar, 5, x, b, n, C), a, d, w, eps=1e-7 if near else 1e-6)
        assert abs(vjp @ d - ref) < 1e-7 * (abs(ref) + np.abs(vjp).max() * np.abs(d).max()), (vjp @ d, ref)


@pytest.mark.parametrize("near", [False, True])
def test_chandrashekar_vjp_both_arguments(pw, near):
    """The one-sweep VJP with respect to both states: each side against central
    differences in that state, and the first side equal to the one-sided VJP."""
    rng = np.random.default_rng(3)
    for _ in range(40):
        a = state(rng)
        b = state(rng, 1e-4, a) if near else state(rng)
        n = rng.normal(size=3)
        w = rng.normal(size=5)
        Uab, Ubb = np.zeros(5), np.zeros(5)
        pw.pw_chandrashekar_vjp_ab(P(a), P(b), P(n), P(C), P(w), P(Uab), P(Ubb))
        one = call(pw.pw_chandrashekar_vjp_a, 5, a, b, n, C, w)
        assert np.allclose(Uab, one, rtol=1e-12, atol=1e-12 * np.abs(one).max())
        eps = 1e-7 if near else 1e-6
        da = rng.normal(size=5) * np.abs(a)
        db = rng.normal(size=5) * np.abs(b)
        ref_a = fd_dot(lambda x: call(pw.pw_chandrashekar, 5, x, b, n, C), a, da, w, eps=eps)
        ref_b = fd_dot(lambda x: call(pw.pw_chandrashekar, 5, a, x, n, C), b, db, w, eps=eps)
        assert abs(Uab @ da - ref_a) < 1e-7 * (abs(ref_a) + np.abs(Uab).max() * np.abs(da).max())
        assert abs(Ubb @ db - ref_b) < 1e-7 * (abs(ref_b) + np.abs(Ubb).max() * np.abs(db).max())


def test_euler_and_viscous_vjp(pw):
    rng = np.random.default_rng(2)
    for _ in range(40):
        U = state(rng)
        n = rng.normal(size=3)
        w = rng.normal(size=5)
        d = rng.normal(size=5)
        vjp = call(pw.pw_euler_flux_vjp, 5, U, n, C, w)
        ref = fd_dot(lambda x: call(pw.pw_euler_flux, 5, x, n, C), U, d, w)
        assert abs(vjp @ d - ref) < 1e-8 * (1 + abs(ref))
        g = rng.normal(size=12)
        wg = rng.normal(size=4)
        gb, Ub = np.zeros(12), np.zeros(5)
        pw.pw_viscous_flux_vjp(P(U), P(g), P(n), P(C), P(wg), P(gb), P(Ub))
        dg = rng.normal(size=12)
        ref_g = fd_dot(lambda x: call(pw.pw_viscous_flux, 4, U, x, n, C), g, dg, wg)
        assert abs(gb @ dg - ref_g) < 1e-8 * (1 + abs(ref_g))
        ref_U = fd_dot(lambda x: call(pw.pw_viscous_flux, 4, x, g, n, C), U, d, wg)
        assert abs(Ub @ d - ref_U) < 1e-8 * (1 + abs(ref_U))
        qb = rng.normal(size=4)
        vq = call(pw.pw_qvars_vjp, 5, U, C, qb)
        ref_q = fd_dot(lambda x: call(pw.pw_qvars, 4, x, C), U, d, qb)
        assert abs(vq @ d - ref_q) < 1e-8 * (1 + abs(ref_q))


@pytest.mark.parametrize("law", [0, 1])
def test_viscous_tensor_vjp(pw, law):
    """One adjoint of the whole viscous flux tensor with weights M[d][v] (the
    adjoint residual sums its three directions' weights into one M) against
    central differences of sum_d M[d] . G(n = e_d), constant and Sutherland."""
    rng = np.random.default_rng(5 + law)
    c = C.copy()
    c[6] = law
    E = np.eye(3)
    for _ in range(30):
        U = state(rng)
        g = rng.normal(size=12)
        M = rng.normal(size=(3, 4))
        gb, Ub = np.zeros(12), np.zeros(5)
        pw.pw_viscous_tensor_vjp(P(U), P(g), P(M), P(c), P(gb), P(Ub))

        def fwd(Ux, gx):
            return sum(M[d] @ call(pw.pw_viscous_flux, 4, Ux, gx, E[d], c) for d in range(3))

        dg, dU = rng.normal(size=12), rng.normal(size=5)
        eps = 1e-6
        ref_g = (fwd(U, g + eps * dg) - fwd(U, g - eps * dg)) / (2 * eps)
        ref_U = (fwd(U + eps * dU, g) - fwd(U - eps * dU, g)) / (2 * eps)
        assert abs(gb @ dg - ref_g) < 1e-8 * (1 + abs(ref_g))
        assert abs(Ub @ dU - ref_U) < 1e-8 * (1 + abs(ref_U))


@pytest.mark.parametrize("form,phys", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("riemann", [0, 1])
def test_surface_flux_vjp(pw, form, phys, riemann):
    rng = np.random.default_rng(3 + form + 2 * phys)
    c = C.copy()
    c[4] = riemann
    for it in range(40):
        UL = state(rng)
        UR = state(rng, 1e-5, UL) if it % 3 == 0 else state(rng)
        if it % 5 == 1:
            UR = UL.copy()
            UR[1:4] *= -1.0          # equal wave speeds on both sides: tie goes to the master side
            UR = UR * (1 + 1e-3 * rng.uniform(-1, 1, 5))
        gL, gR = rng.normal(size=12), rng.normal(size=12)
        nh = rng.normal(size=3)
        nh /= np.linalg.norm(nh)
        s = rng.uniform(0.5, 2.0)
        w = rng.normal(size=5)
        ULb, URb, gLb, gRb = np.zeros(5), np.zeros(5), np.zeros(12), np.zeros(12)
        pw.pw_surface_flux_vjp(form, phys, P(UL), P(UR), P(gL), P(gR), P(nh), ctypes.c_double(s), P(c), P(w),
                               P(ULb), P(URb), P(gLb), P(gRb))

        def fwd(UL_, UR_, gL_, gR_):
            out = np.zeros(5)
            pw.pw_surface_flux(form, phys, P(UL_), P(UR_), P(gL_), P(gR_), P(nh), ctypes.c_double(s), P(c), P(out))
            return out

        dL, dR, dgL, dgR = (rng.normal(size=k) for k in (5, 5, 12, 12))
        eps = 1e-7
        ref = w @ ((fwd(UL + eps * dL, UR + eps * dR, gL + eps * dgL, gR + eps * dgR) -
                    fwd(UL - eps * dL, UR - eps * dR, gL - eps * dgL, gR - eps * dgR)) / (2 * eps))
        got = ULb @ dL + URb @ dR + (gLb @ dgL + gRb @ dgR if phys else 0.0)
        assert abs(got - ref) < 1e-6 * (1 + abs(ref)), (it, got, ref)


def test_fp32_reference_state_rounds_deviations_only(pw):
    """Low-Mach pairs (p ~ 71, small jumps): the float two-point and advective
    fluxes about the reference state (p0, 2 p0/rho0) keep the momentum and
    energy error near float rounding of the deviations, far below the float
    evaluation without a reference state; the reference changes rounding only."""
    rng = np.random.default_rng(31)
    p0 = 1.0 / (G * 0.01)
    ref, none = np.array([p0, 2.0 * p0]), np.array([0.0, 0.0])
    e_ref, e_none, ea_ref, ea_none = [], [], [], []
    for _ in range(500):
        def st():
            rho = 1 + 0.01 * rng.uniform(-1, 1)
            u = rng.uniform(-1, 1, 3)
            p = p0 + rng.uniform(-1, 1)
            return np.array([rho, *(rho * u), p / (G - 1) + 0.5 * rho * u @ u])
        a = st()
        b = a + 0.01 * (st() - a)
        n = rng.normal(size=3)
        F = call(pw.pw_chandrashekar, 5, a, b, n, C)
        e_ref.append(np.abs(call(pw.pw_chandrashekar_f32_ref, 5, a, b, n, C, ref) - F))
        e_none.append(np.abs(call(pw.pw_chandrashekar_f32_ref, 5, a, b, n, C, none) - F))
        E = call(pw.pw_euler_flux, 5, a, n, C)
        ea_ref.append(np.abs(call(pw.pw_euler_flux_f32_ref, 5, a, n, C, ref) - E))
        ea_none.append(np.abs(call(pw.pw_euler_flux_f32_ref, 5, a, n, C, none) - E))
    e_ref, e_none = np.max(e_ref, 0), np.max(e_none, 0)
    ea_ref, ea_none = np.max(ea_ref, 0), np.max(ea_none, 0)
    assert np.all(e_ref[1:4] < 1e-6) and e_ref[4] < 1e-5, e_ref
    assert np.all(e_ref[1:] * 20 < e_none[1:]), (e_ref, e_none)
    assert np.all(ea_ref[1:] < 2e-6) and np.all(ea_ref[1:] * 10 < ea_none[1:]), (ea_ref, ea_none)


def test_entropy_projection_vjps(pw):
    """The adjoints of the two maps of the entropy projection, v(U) and its
    inverse u(v), against central differences of the forward maps, and the
    inverse pair round trip."""
    rng = np.random.default_rng(41)
    for _ in range(20):
        U = state(rng)
        v = call(pw.pw_entropy_vars, 5, U, C)
        assert np.allclose(call(pw.pw_entropy_to_cons, 5, v, C), U, rtol=1e-12, atol=1e-12)
        d, w = rng.normal(size=5), rng.normal(size=5)
        ref = fd_dot(lambda x: call(pw.pw_entropy_vars, 5, x, C), U, d, w, eps=1e-7)
        assert abs(call(pw.pw_entropy_vars_vjp, 5, U, C, w) @ d - ref) < 1e-7 * (1 + abs(ref))
        ref = fd_dot(lambda x: call(pw.pw_entropy_to_cons, 5, x, C), v, d, w, eps=1e-7)
        assert abs(call(pw.pw_entropy_to_cons_vjp, 5, v, C, w) @ d - ref) < 1e-7 * (1 + abs(ref))

