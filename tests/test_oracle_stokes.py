"""Pins of the oracle's Stokes conversion (Section 2.1: instrumental-polarisation images to
Stokes parameters by a per-pixel 4 x 4 matrix that depends on time and sky position; Table
1, "Stokes Conversion"). Nothing here re-types the oracle's Kronecker-product formula: the
pins are a hand-worked pixel, a forward model written with 2 x 2 coherency matrices
(measured = J C J^H, the definition of the instrument's response) whose inversion must
recover the Stokes parameters, the linear-feed special cases, and linearity."""
import numpy as np
import pytest


def test_hand_worked_pixel_ideal_feeds(orc):
    # XX = I + Q, YY = I - Q, XY = U + iV, YX = U - iV (linear feeds). Images as gridded
    # without the Hermitian mirror: the full instrumental image adds the conjugate image, so
    # XX counts twice its real part, and XY gains conj(YX).
    z = np.zeros((4, 1, 1), dtype=np.complex128)
    z[0] = 0.75 + 0.3j   # 2 Re XX = 1.5 = I + Q
    z[3] = 0.25 - 0.7j   # 2 Re YY = 0.5 = I - Q
    z[1] = 0.25 + 0.1j   # XY + conj(YX) = 0.5 + 0.2j = U + iV
    z[2] = 0.25 - 0.1j
    s = orc.stokes(z)[:, 0, 0]
    np.testing.assert_allclose(s, [1.0, 0.5, 0.5, 0.2], rtol=0, atol=1e-15)


def test_xx_only_is_half_i_half_q(orc):
    z = np.zeros((4, 1, 1), dtype=np.complex128)
    z[0] = 1.0  # full XX = 2: I + Q = 2, I - Q = 0
    np.testing.assert_allclose(orc.stokes(z)[:, 0, 0], [1.0, 1.0, 0.0, 0.0], atol=1e-15)


def _random_jones(rng, shape):
    J = rng.standard_normal(shape + (2, 2)) + 1j * rng.standard_normal(shape + (2, 2))
    J += 2.0 * np.eye(2)  # well conditioned
    return J


def test_round_trip_through_a_forward_instrument_model(orc):
    rng = np.random.default_rng(5)
    ny, nx = 6, 7
    I = rng.uniform(1.0, 3.0, (ny, nx))
    Q, U, V = (rng.uniform(-0.5, 0.5, (ny, nx)) for _ in range(3))
    J = _random_jones(rng, (ny, nx))
    z = np.zeros((4, ny, nx), dtype=np.complex128)
    for y in range(ny):
        for x in range(nx):
            C = np.array([[I[y, x] + Q[y, x], U[y, x] + 1j * V[y, x]],
                          [U[y, x] - 1j * V[y, x], I[y, x] - Q[y, x]]])
            Cm = J[y, x] @ C @ J[y, x].conj().T
            # unmirrored images whose mirror completion gives Cm: half the (real) diagonal,
            # the whole of XY and nothing in YX
            z[0, y, x] = Cm[0, 0].real / 2 + 0.37j
            z[3, y, x] = Cm[1, 1].real / 2 - 0.11j
            z[1, y, x] = Cm[0, 1]
            z[2, y, x] = 0.0
    s = orc.stokes(z, jones=J)
    for got, want in zip(s, (I, Q, U, V)):
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_parallactic_rotation_turns_q_into_u(orc):
    # Feeds rotated by an angle chi on the sky: a source of pure Q = 1 appears as
    # Q' = cos 2chi, U' = -sin 2chi in the feed frame; undoing the rotation recovers Q.
    chi = 0.3
    R = np.array([[np.cos(chi), np.sin(chi)], [-np.sin(chi), np.cos(chi)]])
    C = np.array([[2.0, 0.0], [0.0, 0.0]])  # I = Q = 1
    Cm = R @ C @ R.T
    z = np.zeros((4, 1, 1), dtype=np.complex128)
    z[0, 0, 0] = Cm[0, 0] / 2
    z[3, 0, 0] = Cm[1, 1] / 2
    z[1, 0, 0] = Cm[0, 1]
    feed = orc.stokes(z)[:, 0, 0]
    np.testing.assert_allclose(feed, [1.0, np.cos(2 * chi), -np.sin(2 * chi), 0.0], atol=1e-15)
    sky = orc.stokes(z, jones=np.broadcast_to(R, (1, 1, 2, 2)))[:, 0, 0]
    np.testing.assert_allclose(sky, [1.0, 1.0, 0.0, 0.0], atol=1e-14)


def test_linearity_and_pixel_subset(orc):
    rng = np.random.default_rng(6)
    a = rng.standard_normal((4, 5, 4)) + 1j * rng.standard_normal((4, 5, 4))
    b = rng.standard_normal((4, 5, 4)) + 1j * rng.standard_normal((4, 5, 4))
    J = _random_jones(rng, (5, 4))
    sa, sb = orc.stokes(a, J), orc.stokes(b, J)
    np.testing.assert_allclose(orc.stokes(2.0 * a - 3.0 * b, J), 2.0 * sa - 3.0 * sb, atol=1e-12)
    pix = np.array([[0, 0], [3, 4], [1, 2]])
    np.testing.assert_allclose(orc.stokes(a, J, pixels=pix), sa[:, pix[:, 1], pix[:, 0]], atol=0)


def test_identity_jones_equals_ideal_feeds(orc):
    rng = np.random.default_rng(7)
    a = rng.standard_normal((4, 3, 3)) + 1j * rng.standard_normal((4, 3, 3))
    J = np.broadcast_to(np.eye(2, dtype=np.complex128), (3, 3, 2, 2))
    np.testing.assert_allclose(orc.stokes(a, J), orc.stokes(a), atol=1e-15)
