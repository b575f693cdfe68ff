"""Pin of the absorbing base, the base input force and the layered medium
(Sections 2-3: input velocity applied as a force at the base,
semi-infinite absorbing boundary) against the closed-form transfer function
of one soft layer on an elastic half-space for vertically incident SH waves:

    |V_surf / V_inc| = 2 / |cos(k1 H) + i a sin(k1 H)|,
    k1 = w / Vs1,  a = rho1 Vs1 / (rho2 Vs2).

The oracle models a column one cell wide, motion along x1 only (x2, x3
displacements held at zero), no side dashpots, base dashpot plus the
incident-wave force 2 rho2 Vs2 v_in, no damping.  The continuum solution of
that column is the 1D one, so the FE result must approach the closed form
as h and dt shrink."""
import numpy as np
import pytest

import casegen as cg
from oracle import march

H, DEPTH = 20.0, 40.0


def _transfer(h, dt, T=12.0, fp=2.0):
    mesh = cg.box_mesh(h, h, DEPTH, h)
    mat = cg.material_table()
    c = cg.tet_centroids(mesh)
    tet_mat = np.where(-c[:, 2] < H, 0, 1).astype(np.uint8)
    n = int(round(T / dt))
    v_in = cg.incident_velocity(n, dt, (fp,), 1.0 / fp)
    case = cg.Case(mat=mat, tet_mat=tet_mat, rec_node=np.array([0], np.int32), v_in=v_in,
                   dt=dt, n_steps=n, ray_alpha=0.0, ray_beta=0.0)
    sys = march.build_system(mesh, case, damping=False, dashpot_roles=(2,))
    top = np.nonzero(np.abs(mesh.xyz[:, 2]) < 1e-9)[0]
    nn = np.arange(mesh.n_nodes)
    fixed = np.concatenate([3 * nn + 1, 3 * nn + 2])
    r = march.run(sys, dt, v_in, n, top, fixed_dofs=fixed)
    v_top = r.rec_v[:, :, 0]
    vs = np.concatenate([[0.0], v_top.mean(1)])
    nf = 8 * len(vs)
    f = np.fft.rfftfreq(nf, dt)
    R = np.abs(np.fft.rfft(vs, nf)) / np.abs(np.fft.rfft(v_in[:, 0], nf))
    s1, s2 = mat[0], mat[1]
    k1 = 2 * np.pi * f / s1[1]
    a = s1[2] * s1[1] / (s2[2] * s2[1])
    th = 2 / np.abs(np.cos(k1 * H) + 1j * a * np.sin(k1 * H))
    band = (f >= 0.2) & (f <= 2.5)
    err = np.max(np.abs(R[band] - th[band]) / th[band])
    spread = np.abs(v_top - v_top.mean(1, keepdims=True)).max() / np.abs(v_top).max()
    return err, spread, R[band].max(), th[band].max()


def test_sh_layer_transfer_function():
    err, spread, peak, th_peak = _transfer(2.0, 0.005)
    assert err < 0.005                       # well inside 2 %
    assert abs(th_peak - 2 / 0.27) < 2e-3    # the band reaches the resonance peak 2/a
    assert abs(peak - th_peak) < 0.005 * th_peak
    assert spread < 1e-3


def test_sh_transfer_converges_in_time_and_space():
    e1, s1, _, _ = _transfer(4.0, 0.005)
    e2, _, _, _ = _transfer(4.0, 0.0025)
    _, s3, _, _ = _transfer(10.0, 0.005)
    assert e2 < 0.5 * e1          # second-order time integrator
    assert s1 < 0.2 * s3          # departure from the 1D motion shrinks with h


@pytest.mark.parametrize("wrong", ["no_factor_two", "p_impedance"])
def test_sh_closed_form_rejects_planted_mistakes(wrong, monkeypatch):
    # A plausible mistake in the base force or dashpot must fail the pin:
    # plant it in the oracle (on the CPU) and check the error is large.
    from oracle import assemble, fem
    if wrong == "no_factor_two":
        orig = assemble.input_force_basis
        monkeypatch.setattr(assemble, "input_force_basis", lambda *a: 0.5 * orig(*a))
    else:
        orig = fem.face_impedance
        monkeypatch.setattr(fem, "face_impedance", lambda n, vp, vs, rho: orig(n, vp, vp, rho))
    err, _, _, _ = _transfer(4.0, 0.005, T=8.0)
    assert err > 0.05
