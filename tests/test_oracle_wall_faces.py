"""Magnetic faces on a PEC wall (our reading of Sec. 2 and 3.2.2, which
evolve M where the magnetic material meets the field): the wall holds normal
B, so a wall face's normal H stays 0 and its M is not evolved.  Its M0 is
the value of the one cell beside it (the two-cell face mean with the wall
side clamped), along m0 and of length Ms.  Checked on a magnetised block
against the x = 0 wall, driven hard, while the interior faces of the same
block move."""
import numpy as np

from oracle import Simulation

N = (12, 6, 5)
D = (1e-4, 1e-4, 1e-4)


def _block_sim():
    nx, ny, nz = N
    Ms = np.zeros((nz, ny, nx))          # host layout [k][j][i]
    Ms[:, :, :4] = 1.4e5                 # cells 0-3 along x: against the x = 0 wall
    Ms[:, :, 2] = 1.75e5
    m = np.array([0.3, 0.2, 0.93])
    m0 = np.stack([np.full((nz, ny, nx), v) for v in m])
    alpha = np.full((nz, ny, nx), 0.01)
    dt = 0.5 * D[0] / (3e8 * np.sqrt(3))
    sim = Simulation(N, D, dt, Ms=Ms, alpha=alpha, m0_dir=m0, H0=(0.0, 0.0, 2.0e5))
    rng = np.random.default_rng(7)
    E = [rng.standard_normal(sim.E[c].shape) * 3e3 for c in range(3)]
    H = [rng.standard_normal(sim.H[c].shape) * 3e2 for c in range(3)]
    for c in range(3):
        sim.E[c] = np.where(sim.e_interior[c], E[c], 0.0)
        sim.H[c] = np.where(sim.h_interior[c], H[c], 0.0)
    return sim, m / np.linalg.norm(m)


def test_wall_faces_hold_m0_and_zero_normal_h():
    sim, mhat = _block_sim()
    wall = sim.mag[0] & ~sim.h_interior[0]       # x faces on the x = 0 wall
    inner = sim.evolve[0]
    assert wall[0].all() and not wall[1:].any()   # the whole i = 0 plane, nothing else
    assert inner[1:4].all()
    M0 = [v.copy() for v in sim.M[0]]
    # M0 on a wall face: Ms of the one cell beside it, along m0
    for c in range(3):
        assert np.allclose(M0[c][0], 1.4e5 * mhat[c], rtol=1e-14, atol=0)
    sim.step(20)
    for c in range(3):
        assert np.array_equal(sim.M[0][c][wall], M0[c][wall])
        assert np.max(np.abs(sim.M[0][c][inner] - M0[c][inner])) > 1e-6 * 1.4e5
    assert np.all(sim.H[0][0] == 0)
    # |M| = Ms on every magnetic face, wall faces included
    for f in range(3):
        nrm = np.sqrt(sum(sim.M[f][c] ** 2 for c in range(3)))
        mag = sim.mag[f]
        assert np.allclose(nrm[mag], sim.Ms_f[f][mag], rtol=1e-12, atol=0)
