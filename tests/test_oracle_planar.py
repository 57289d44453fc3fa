"""Pins of the node-centred CIC density and of the plane-parallel reduction.

Both serve the full-size (1024^3) parity tests, where the oracle evaluates
sampled outputs one by one.  Each is pinned against the independent 3-D oracle
(corner-enumerated CIC deposit; 3-D Fourier solve, gather, kick and drift) on
small meshes, where the two must agree to rounding."""
import pytest
import torch

import synth_inputs as si
from oracle import cic, cosmology as ocm, integrate, planar, solve


def test_rho_at_nodes_equals_corner_deposit():
    n = 8
    x = torch.from_numpy(si.uniform_particles(n, 300, 4))
    rho = cic.deposit_rho(x, n)
    g = torch.arange(n)
    nodes = torch.stack(torch.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    got = cic.rho_at_nodes(nodes, x, n)
    assert torch.allclose(got, rho.reshape(-1), atol=1e-12)
    assert float(got.sum()) == pytest.approx(300.0, rel=1e-13)


def test_rho_at_nodes_wraps_and_ignores_far_particles():
    n = 16
    # a particle at 15.25 along x shares its weight between nodes 15 (0.75) and 0 (0.25)
    x = torch.tensor([[15.25, 7.0], [3.0, 7.0], [4.0, 7.0]], dtype=torch.float64)
    nodes = torch.tensor([[15, 0, 14, 7], [3, 3, 3, 7], [4, 4, 4, 7]])
    got = cic.rho_at_nodes(nodes, x, n)
    assert got.tolist() == pytest.approx([0.75, 0.25, 0.0, 1.0], abs=1e-15)


def _planar_case(n, axis, seed, offset):
    coord, mom = si.planar_profile(n, axis, seed, amp_log2=1, mom_log2=-1)
    coord[(axis + 1) % 3] = offset
    c = coord.double() * si.QUANTUM
    m = mom.double() * si.QUANTUM
    pos, p3 = si.expand_planar(coord, mom, n, axis, dtype=torch.float64)
    return c, m, pos, p3


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("grad", ["spectral", "fd2", "fd1"])
def test_planar_cycle_equals_3d_oracle(axis, grad):
    n = 16
    om = ocm.FIDUCIAL.omega_m
    c, m, pos, p3 = _planar_case(n, axis, 20 + axis, 3 * 8192 + 77)
    kick, drift = 0.8, 1.7
    c1, m1, f1 = planar.cycle_line(c, m, axis, kick, drift, n, om, grad)

    meshes = solve.newton_forces(cic.deposit_delta(pos, n), om, grad)
    want = torch.zeros_like(meshes)
    shape = [1, 1, 1]
    shape[axis] = n
    want[axis] = f1.view(shape).expand(n, n, n)
    assert torch.allclose(meshes, want, atol=1e-12)

    wx, wv = integrate.force_then_kick_drift(pos, p3, kick, drift, integrate.NewtonForce(n, grad=grad), 0.0, n)
    g = torch.arange(n)
    q = torch.stack(torch.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    got_x = planar.particle_coords(c1, axis, n, q)
    d = torch.remainder(got_x - wx + n / 2, n) - n / 2
    assert float(d.abs().max()) < 1e-12
    assert torch.allclose(m1[:, q[axis]], wv, atol=1e-12)


def test_planar_density_is_mass_conserving_and_uniform_lattice_is_force_free():
    n = 32
    om = ocm.FIDUCIAL.omega_m
    x = torch.arange(n, dtype=torch.float64) + 0.5
    assert torch.allclose(planar.deposit_delta_line(x, n), torch.zeros(n, dtype=torch.float64), atol=1e-15)
    coord, _ = si.planar_profile(n, 0, 3)
    d = planar.deposit_delta_line(coord[0].double() * si.QUANTUM, n)
    assert abs(float(d.sum())) < 1e-12
    assert float(planar.newton_force_line(d, om).sum()) == pytest.approx(0.0, abs=1e-12)
