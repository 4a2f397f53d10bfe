"""Pins of the oracle's pointwise numerics against facts independent of the oracle.

WENO5-JS (Jiang & Shu, cited in the paper's "Numerical Scheme"): exact for quadratics
whatever the weights; reduces to the linear fifth-order upwind formula on smooth data;
ENO behaviour at a step.  Roe eigen-system: L R = I, the Roe property
A(uR-uL) = f(uR)-f(uL), and the analytic Jacobian for uL = uR.  Face flux: consistency,
upwind stencil independence, mirror symmetry.  SSP-RK3: stability polynomial.
"""
import numpy as np
import pytest

GAMMA = 1.4


def cons(rho, u, v, w, p, gamma=GAMMA, B=0.0):
    return np.array([rho, rho * u, rho * v, rho * w,
                     (p + gamma * B) / (gamma - 1) + 0.5 * rho * (u * u + v * v + w * w)])


def flux_independent(U, gamma=GAMMA, B=0.0):
    """Euler flux along x written from its textbook definition (not the oracle's code)."""
    rho, mx, my, mz, E = U
    u = mx / rho
    p = (gamma - 1) * (E - 0.5 * (mx * mx + my * my + mz * mz) / rho) - gamma * B
    return np.array([mx, mx * u + p, my * u, mz * u, (E + p) * u])


def test_pressure_and_flux(orc):
    rng = np.random.default_rng(0)
    for _ in range(20):
        rho, p = rng.uniform(0.1, 3, 2)
        u, v, w = rng.normal(size=3)
        B = rng.uniform(0, 2)
        U = cons(rho, u, v, w, p, B=B)
        assert abs(orc.pressure(U, GAMMA, B) - p) <= 1e-13 * (1 + p)
        np.testing.assert_allclose(orc.flux_x(U, GAMMA, B), flux_independent(U, B=B), rtol=1e-14, atol=1e-14)


def test_weno_exact_for_quadratics(orc):
    # Cell averages of q(x) = a + b x + c x^2 on unit cells centred at -2..2: every
    # candidate polynomial reproduces q(1/2) exactly, so the result does for any weights.
    rng = np.random.default_rng(1)
    for _ in range(50):
        a, b, c = rng.normal(size=3) * rng.choice([1e-3, 1.0, 1e3])
        avg = [a + b * x + c * (x * x + 1.0 / 12.0) for x in (-2, -1, 0, 1, 2)]
        exact = a + b * 0.5 + c * 0.25
        got = orc.weno5_minus(*avg)
        assert abs(got - exact) <= 1e-12 * (abs(a) + abs(b) + abs(c))


def test_weno_linear_limit(orc):
    # beta << eps_w: nonlinear weights -> (0.1, 0.6, 0.3), i.e. (2,-13,47,27,-3)/60.
    rng = np.random.default_rng(2)
    for _ in range(50):
        f = rng.normal(size=5) * 1e-6
        lin = (2 * f[0] - 13 * f[1] + 47 * f[2] + 27 * f[3] - 3 * f[4]) / 60.0
        got = orc.weno5_minus(*f)
        assert abs(got - lin) <= 1e-4 * np.abs(f).max()


def test_weno_eno_at_step(orc):
    # A jump between d and e: the smooth candidate (a,b,c) dominates, result ~ c.
    got = orc.weno5_minus(0.0, 0.0, 0.0, 0.0, 1.0)
    assert abs(got) < 1e-9
    got = orc.weno5_minus(1.0, 1.0, 1.0, 0.0, 0.0)
    assert abs(got - 1.0) < 0.01  # candidate 0 is exactly 1, others are damped


def _random_state(rng, supersonic=None):
    rho, p = rng.uniform(0.2, 2.0), rng.uniform(0.2, 2.0)
    v, w = rng.normal(size=2)
    c = np.sqrt(GAMMA * p / rho)
    if supersonic == "right":
        u = c * rng.uniform(1.2, 2.0)
    elif supersonic == "left":
        u = -c * rng.uniform(1.2, 2.0)
    else:
        u = rng.normal()
    return cons(rho, u, v, w, p)


def test_roe_eigensystem(orc):
    rng = np.random.default_rng(3)
    for _ in range(30):
        UL, UR = _random_state(rng), _random_state(rng)
        R, L = orc.roe_matrices(UL, UR, GAMMA, 0.0)
        np.testing.assert_allclose(L @ R, np.eye(5), atol=1e-12)
        # Eigenvalues read off the eigenvectors: R[1, :] = (u-c, u, v?, ...) ->
        # R[1,1] = u, R[1,4] - R[1,1] = c.
        u, c = R[1, 1], R[1, 4] - R[1, 1]
        A = R @ np.diag([u - c, u, u, u, u + c]) @ L
        dU = UR - UL
        df = flux_independent(UR) - flux_independent(UL)
        np.testing.assert_allclose(A @ dU, df, rtol=1e-11, atol=1e-11 * np.abs(df).max())


def test_roe_matrix_equals_jacobian(orc):
    rng = np.random.default_rng(4)
    for _ in range(10):
        U = _random_state(rng)
        R, L = orc.roe_matrices(U, U, GAMMA, 0.0)
        u, c = R[1, 1], R[1, 4] - R[1, 1]
        # speed of sound from the state, independently
        rho = U[0]
        p = (GAMMA - 1) * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho)
        assert abs(c - np.sqrt(GAMMA * p / rho)) < 1e-12
        A = R @ np.diag([u - c, u, u, u, u + c]) @ L
        J = np.zeros((5, 5))
        for k in range(5):
            h = 1e-6 * max(1.0, abs(U[k]))
            e = np.zeros(5)
            e[k] = h
            J[:, k] = (flux_independent(U + e) - flux_independent(U - e)) / (2 * h)
        np.testing.assert_allclose(A, J, atol=1e-6)


@pytest.mark.parametrize("kind", [None, "right", "left"])
def test_face_flux_consistency(orc, kind):
    rng = np.random.default_rng(5)
    for d in range(3):
        for _ in range(10):
            U = _random_state(rng, kind)
            # rotate the velocity so that the chosen supersonic component is along axis d
            Ud = U.copy()
            Ud[1 + d], Ud[1] = U[1], U[1 + d]
            st = np.tile(Ud, (6, 1))
            F, _ = orc.face_flux(d, st)
            # physical flux along axis d, from the definition
            rho = Ud[0]
            vel = Ud[1:4] / rho
            p = (GAMMA - 1) * (Ud[4] - 0.5 * rho * vel @ vel)
            f = np.array([Ud[1 + d], *(Ud[1:4] * vel[d]), (Ud[4] + p) * vel[d]])
            f[1 + d] += p
            np.testing.assert_allclose(F, f, rtol=1e-12, atol=1e-12)


def test_face_flux_upwind_stencil(orc):
    # Supersonic to the right: all eigenvalues of both face cells positive -> the flux
    # uses cells i-2..i+2 only; the downwind-most cell (index 5) must not matter.
    rng = np.random.default_rng(6)
    for _ in range(10):
        base = _random_state(rng, "right")
        st = np.array([base * (1 + 0.01 * rng.normal()) for _ in range(6)])
        # keep it supersonic: scale momentum up
        st[:, 1] *= 1.0
        F1, n1 = orc.face_flux(0, st)
        st2 = st.copy()
        st2[5] = _random_state(rng)
        F2, _ = orc.face_flux(0, st2)
        assert n1 == 0
        assert np.array_equal(F1, F2)
    for _ in range(10):
        base = _random_state(rng, "left")
        st = np.array([base * (1 + 0.01 * rng.normal()) for _ in range(6)])
        F1, n1 = orc.face_flux(0, st)
        st2 = st.copy()
        st2[0] = _random_state(rng)
        F2, _ = orc.face_flux(0, st2)
        assert n1 == 0
        assert np.array_equal(F1, F2)


def test_face_flux_llf_branch_uses_all_cells(orc):
    # Normal velocity changes sign across the face: the u-fields take the LLF branch,
    # whose W+ half reads the downwind-most cell.
    rng = np.random.default_rng(7)
    st = np.array([cons(1 + 0.1 * rng.normal(), 0.05 * rng.normal(), 0.1, -0.2,
                        1 + 0.1 * rng.normal()) for _ in range(6)])
    st[2] = cons(1.0, 0.05, 0.1, -0.2, 1.0)
    st[3] = cons(1.1, -0.05, 0.1, -0.2, 1.05)
    F1, n = orc.face_flux(0, st)
    assert n == 3
    st2 = st.copy()
    st2[5] = cons(1.5, -0.03, 0.3, 0.1, 1.2)
    F2, _ = orc.face_flux(0, st2)
    assert not np.array_equal(F1, F2)


def test_face_flux_mirror_symmetry(orc):
    # Reflection x -> -x: reverse the stencil, negate the normal momentum; the flux of
    # rho, rho v, rho w, E changes sign and the normal momentum flux does not.
    rng = np.random.default_rng(8)
    for _ in range(20):
        st = np.array([_random_state(rng) for _ in range(6)])
        F, _ = orc.face_flux(0, st)
        mir = st[::-1].copy()
        mir[:, 1] *= -1
        Fm, _ = orc.face_flux(0, mir)
        expect = np.array([-F[0], F[1], -F[2], -F[3], -F[4]])
        np.testing.assert_allclose(Fm, expect, rtol=1e-11, atol=1e-11 * np.abs(F).max())


def test_ssprk3_stability_polynomial(orc):
    # u' = lam u: three stages reproduce 1 + z + z^2/2 + z^3/6, z = lam dt.
    for z in (-0.5, -1.0, 0.3, -2.0):
        dt, lam, u0 = 0.1, z / 0.1, 1.7
        u1 = orc.ssprk3_stage(0, u0, u0, lam * u0, dt)
        u2 = orc.ssprk3_stage(1, u0, u1, lam * u1, dt)
        u3 = orc.ssprk3_stage(2, u0, u2, lam * u2, dt)
        assert abs(u3 - u0 * (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-14
