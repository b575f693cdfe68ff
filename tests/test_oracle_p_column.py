"""Pin of the compressional half of the oracle: the Lame constant lambda,
the normal (rho Vp) term of the absorbing dashpot and the vertical
component (2 rho Vp) of the base input force (Section 2, Eq. GE:ORG with
the semi-infinite absorbing base; Section 3, input applied as forces from
the bottom).  The shear half is pinned by the SH column test.

A column one cell wide with x1 and x2 displacements held at zero deforms
in uniaxial strain, whose modulus is lambda + 2 mu = rho Vp^2: a vertically
incident P wave in a soft layer of thickness H over an elastic half-space
then has the closed-form surface transfer function

    |V_surf / V_inc| = 2 / |cos(k1 H) + i a sin(k1 H)|,
    k1 = w / Vp1,  a = rho1 Vp1 / (rho2 Vp2).

The base carries the normal dashpot rho2 Vp2 and the force 2 rho2 Vp2 v_in,3;
no side dashpots, no damping.  The materials are slower than the benchmark
layers so that the layer resonance Vp1 / (4 H) = 3.75 Hz lies inside the
band of the input (the benchmark soft layer would put it at 20 Hz, where a
2 Hz input has no energy and the transfer function is nearly flat)."""
import numpy as np
import pytest

import casegen as cg
from oracle import assemble, fem, march

H, DEPTH = 20.0, 40.0
SOFT_P = (300.0, 150.0, 1800.0)    # Vp, Vs, rho
ROCK_P = (1000.0, 500.0, 2000.0)   # a = 1800 * 300 / (2000 * 1000) = 0.27
BAND = (0.5, 6.0)                  # Hz


def _transfer(h, dt, T=8.0, fp=4.0):
    mesh = cg.box_mesh(h, h, DEPTH, h)
    mat = np.array([SOFT_P, ROCK_P])
    c = cg.tet_centroids(mesh)
    tet_mat = np.where(-c[:, 2] < H, 0, 1).astype(np.uint8)
    n = int(round(T / dt))
    v_in = cg.incident_velocity(n, dt, (fp,), 1.0 / fp, direction=2)
    case = cg.Case(mat=mat, tet_mat=tet_mat, rec_node=np.array([0], np.int32), v_in=v_in,
                   dt=dt, n_steps=n, ray_alpha=0.0, ray_beta=0.0)
    sys = march.build_system(mesh, case, damping=False, dashpot_roles=(2,))
    top = np.nonzero(np.abs(mesh.xyz[:, 2]) < 1e-9)[0]
    nn = np.arange(mesh.n_nodes)
    fixed = np.concatenate([3 * nn, 3 * nn + 1])
    r = march.run(sys, dt, v_in, n, top, fixed_dofs=fixed)
    v_top = r.rec_v[:, :, 2]
    vs = np.concatenate([[0.0], v_top.mean(1)])
    nf = 8 * len(vs)
    f = np.fft.rfftfreq(nf, dt)
    R = np.abs(np.fft.rfft(vs, nf)) / np.abs(np.fft.rfft(v_in[:, 2], nf))
    s1, s2 = mat[0], mat[1]
    k1 = 2 * np.pi * f / s1[0]
    a = s1[2] * s1[0] / (s2[2] * s2[0])
    th = 2 / np.abs(np.cos(k1 * H) + 1j * a * np.sin(k1 * H))
    band = (f >= BAND[0]) & (f <= BAND[1])
    err = np.max(np.abs(R[band] - th[band]) / th[band])
    spread = np.abs(v_top - v_top.mean(1, keepdims=True)).max() / np.abs(v_top).max()
    return err, spread, R[band].max(), th[band].max()


def test_p_layer_transfer_function():
    err, spread, peak, th_peak = _transfer(2.0, 0.005)
    assert err < 0.01                        # measured 0.56 %
    assert abs(th_peak - 2 / 0.27) < 2e-3    # the band reaches the resonance peak 2/a
    assert abs(peak - th_peak) < 0.005 * th_peak
    assert spread < 1e-3


def test_p_transfer_converges_in_time_and_space():
    e_dt1, _, _, _ = _transfer(4.0, 0.005)
    e_dt2, _, _, _ = _transfer(4.0, 0.0025)
    assert e_dt2 < 0.4 * e_dt1               # second-order time integrator (ratio ~4)
    e_h10, _, _, _ = _transfer(10.0, 0.0025)
    e_h5, _, _, _ = _transfer(5.0, 0.0025)
    assert e_h5 < 0.3 * e_h10                # spatial error shrinks with h


def _wrong_vertical_input(orig):
    def f(mesh, mat, tet_mat):
        B = orig(mesh, mat, tet_mat).copy()
        m = tet_mat[mesh.face_tet[mesh.face_role == 2]]
        assert np.all(m == m[0])
        B[2] *= mat[m[0], 1] / mat[m[0], 0]   # 2 rho Vs instead of 2 rho Vp
        return B
    return f


@pytest.mark.parametrize("wrong", ["lambda_rho_vp2", "normal_impedance_vs", "vertical_input_vs"])
def test_p_closed_form_rejects_planted_mistakes(wrong, monkeypatch):
    # A plausible misreading of the compressional terms must fail the pin:
    # plant it in the oracle (on the CPU) and check the error is large.
    if wrong == "lambda_rho_vp2":
        orig = fem.lame

        def lame(mat):
            lam, mu, rho = orig(mat)
            return lam + 2 * mu, mu, rho      # lambda = rho Vp^2
        monkeypatch.setattr(fem, "lame", lame)
    elif wrong == "normal_impedance_vs":
        orig = fem.face_impedance
        monkeypatch.setattr(fem, "face_impedance", lambda n, vp, vs, rho: orig(n, vs, vs, rho))
    else:
        monkeypatch.setattr(assemble, "input_force_basis", _wrong_vertical_input(assemble.input_force_basis))
    err, _, _, _ = _transfer(4.0, 0.005)
    assert err > 0.2                          # measured 0.50 - 0.76
