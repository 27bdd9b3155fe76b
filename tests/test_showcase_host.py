"""Host-side parts of the paper-scale growth-direction runner (no GPU)."""
import numpy as np

from paper_1602_07483_amd import showcase
from paper_1602_07483_amd.inputs import sphere_field


def test_problem_has_the_papers_parameters():
    pb = showcase.problem("k41k61")
    assert (pb.nx, pb.ny, pb.nz) == (351, 351, 351)
    assert (pb.dx, pb.dt, pb.W0, pb.tau0) == (0.01, 1.5e-5, 0.0125, 1.5625e-4)
    assert (pb.lam, pb.kappa, pb.theta0, pb.radius) == (10.0, 1.0, -0.25, 8.0)
    assert (pb.eps, pb.delta, pb.steps) == (0.0, -0.02, 140000)
    assert showcase.problem("cubic").steps == 30000


def test_radii_of_a_corner_sphere():
    """A tanh sphere of radius R centred on the mirror point (-1/2, -1/2, -1/2)
    has its phi = 0 surface at R along every direction."""
    n, R = 40, 17.3
    phi = sphere_field((n, n, n), [(-0.5, -0.5, -0.5)], R, 1.0, 1.0)
    r100, r110, r111 = showcase.radii(phi)
    for r in (r100, r110, r111):
        assert abs(r - R) < 0.05
    assert np.isnan(showcase.outer_crossing(-np.ones(5)))
