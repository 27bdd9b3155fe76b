"""Pins of the oracle through its stored reduction traces (CPU).

The traces under tests/golden/ are written by tests/golden/make_traces.py,
which calls only the oracle.  Here they are (1) checked against numbers the
paper prints and (2) checked to be what the current oracle computes, by
re-running the start of each trace.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1602_07483_amd import inputs
from tests.pairs import make_oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    path = os.path.join(GOLDEN, "trace_%s.json" % name)
    if not os.path.exists(path):
        pytest.skip("trace %s not generated" % name)
    with open(path) as fh:
        return json.load(fh)


def _vp(trace, pb):
    """V_p = V d0 / kappa of each record interval (Sec. 4.1), with the
    record times T = step dt / tau0."""
    steps = np.array([r["step"] for r in trace], dtype=float)
    tips = np.array([r["tip"][0] for r in trace])
    d0 = 0.8839 * pb.W0 / pb.lam                           # a1 W0 / lambda
    v = np.diff(tips) / np.diff(steps) * pb.dx / pb.dt     # W0 / tau0 units
    return steps[1:] * pb.dt / pb.tau0, v * d0 / pb.kappa


def test_thermal2d_tip_velocity_at_the_paper_resolution():
    """Sec. 4.1, anisotropic thermal dendrite at Delta = 0.55, delta x/W0 =
    0.4, T = 300, as a one-node D3Q19 slab (D2Q9 after the mirror
    reduction): the oracle's V_p is steady (the last third changes by under
    1 %) and symmetric in x and y.  The paper prints V_p = 0.01735 for its
    LB code at this resolution, 0.01667 for its FD/MC code, and quotes the
    sharp-interface Green's-function value 0.0170 and Karma & Rappel's
    0.0174.  The oracle gives 0.01638: 5.6 % below the paper's LB value,
    3.6 % below the Green's-function value.  That gap is discretisation
    error of the scheme at this resolution: under refinement the oracle's
    V_p converges, at first order in delta x, to the Green's-function value
    (test_thermal2d_refinement_converges_to_the_green_function_value)."""
    g = load("thermal2d")
    pb = inputs.workload_thermal2d()
    tr = g["trace"]
    assert tr[-1]["step"] == 37500 and tr[-1]["nonfinite"] == 0
    T, vp = _vp(tr, pb)
    print("V_p(T=300) = %.5f; vs the paper's LB 0.01735 %+.1f %%, FD/MC 0.01667 %+.1f %%, GF 0.0170 %+.1f %%"
          % (vp[-1], 100 * (vp[-1] / 0.01735 - 1), 100 * (vp[-1] / 0.01667 - 1), 100 * (vp[-1] / 0.0170 - 1)))
    late = vp[2 * len(vp) // 3:]
    assert (late.max() - late.min()) / late.mean() < 0.01
    assert abs(tr[-1]["tip"][0] - tr[-1]["tip"][1]) < 1e-9


def test_thermal2d_gradient_stencil_is_not_the_gap():
    """The one discretisation choice left open for the 2D runs, the
    gradient stencil of phi (reading R5, axis central differences), against
    its isotropic lattice variant (oracle grad_stencil = 1): V_p(T = 300)
    agrees within 0.5 %, so the stencil does not explain the 5.6 % gap to the
    paper's LB value."""
    pb = inputs.workload_thermal2d()
    _, va = _vp(load("thermal2d")["trace"], pb)
    g = load("thermal2d_isograd")
    assert g["oracle_options"] == {"skip_U": 1, "grad_stencil": 1}
    _, vi = _vp(g["trace"], pb)
    print("V_p(T=300): axis stencil %.5f, isotropic %.5f" % (va[-1], vi[-1]))
    assert abs(vi[-1] - va[-1]) / va[-1] < 0.005


def test_thermal2d_refinement_converges_to_the_green_function_value():
    """The oracle's V_p under refinement, delta x/W0 = 0.4, 0.3, 0.2 with
    dt proportional to delta x^2 (all relaxation times fixed), seed radius
    4 W0, in a 100 W0 quadrant up to T = 150 (tests/golden/make_traces.py):
    V_p(T = 150) rises monotonically, with successive gains in the ratio of
    an order of convergence between 1 and 2 (ratio 1 for first order, 1.4
    for second at these spacings; observed 1.22, order 1.6).  Extrapolating
    the T = 300 value at delta x/W0 = 0.4 to delta x = 0 with the
    first-order and with the second-order fit of the T = 150 gain brackets
    the converged V_p, and both ends must lie within 1 % of the
    sharp-interface Green's-function value 0.0170 the paper quotes
    (Sec. 4.1): the scheme converges to the right answer and its 3.6 %
    deficit at delta x/W0 = 0.4 is discretisation error."""
    v150 = {}
    for h in (0.4, 0.3, 0.2):
        g = load("thermal2d_dx%g_T150" % h)
        assert g["oracle_options"] == {"skip_U": 1}
        p = g["problem"]
        pb = inputs.workload_thermal2d(n=p["nx"], dx=h)
        assert abs(p["dt"] - pb.dt) < 1e-15 and p["radius"] == pb.radius
        T, vp = _vp(g["trace"], pb)
        assert abs(T[-1] - 150.0) < pb.dt / pb.tau0   # the last whole step before T = 150
        v150[h] = vp[-1]
    d1, d2 = v150[0.3] - v150[0.4], v150[0.2] - v150[0.3]
    slope = (v150[0.2] - v150[0.4]) / 0.2
    _, v300 = _vp(load("thermal2d")["trace"], inputs.workload_thermal2d())
    v0 = v300[-1] + slope * 0.4                                            # first order
    v0_2 = v300[-1] + (v150[0.2] - v150[0.4]) / (0.4 ** 2 - 0.2 ** 2) * 0.4 ** 2   # second order
    print("V_p(T=150) at dx/W0 = 0.4, 0.3, 0.2: %.5f %.5f %.5f; gain ratio %.3f; converged V_p(T=300) "
          "%.5f (first order, %+.2f %% from 0.0170) .. %.5f (second order, %+.2f %%)"
          % (v150[0.4], v150[0.3], v150[0.2], d1 / d2, v0, 100 * (v0 / 0.0170 - 1), v0_2,
             100 * (v0_2 / 0.0170 - 1)))
    assert d1 > 0 and d2 > 0
    assert 0.9 < d1 / d2 < 1.5
    assert abs(v0 - 0.0170) / 0.0170 < 0.01
    assert abs(v0_2 - 0.0170) / 0.0170 < 0.01


@pytest.mark.parametrize("name,factory,steps", [
    ("thermal2d", lambda: inputs.workload_thermal2d(), 500),
    ("octant128", lambda: inputs.workload_octant(128, 5000), 100),
])
def test_trace_start_reproduces(name, factory, steps):
    """The stored trace is what the current oracle computes (first record)."""
    g = load(name)
    pb = factory()
    rec = g["trace"][0]
    assert rec["step"] == steps
    o = make_oracle(pb)
    o.step(steps)
    r = o.reduce(pb.centre())
    for a, key in enumerate((oracle.R_TIPX, oracle.R_TIPY, oracle.R_TIPZ)):
        # no crossing along an axis (the slab's z) is NaN on both sides
        assert np.isclose(r[key], rec["tip"][a], rtol=0, atol=1e-10, equal_nan=True)
    assert abs(r[oracle.R_SOLID] - rec["solid_fraction"]) < 1e-12
    assert abs(r[oracle.R_MASS] - rec["solute_mass"]) < 1e-10 * abs(rec["solute_mass"])
    assert abs(r[oracle.R_ENTHALPY] - rec["enthalpy"]) < 1e-9 * max(1.0, abs(rec["enthalpy"]))


@pytest.mark.parametrize("name", ["fd2d", "fd3d", "fd3d_iso"])
def test_lb_oracle_matches_finite_differences(name):
    """The LB oracle against the independent finite-difference discretisation
    of the same PDEs (oracle/fd_oracle.c), as the paper compares its LB
    schemes with finite differences (Sec. 4): from the same initial fields,
    the phi = 0 tip positions agree within one node at every record and the
    tip velocity of free growth (least-squares slope from a quarter of the
    run until the tip comes within 30 % of the domain of the far wall)
    within 4 %, the spread the paper reports between its own LB and FD/MC
    codes."""
    g = load(name)
    tr = g["trace"]
    n = g["problem"]["nx"]
    steps = np.array([r["step"] for r in tr], dtype=float)
    lb = np.array([r["lb_tip"] for r in tr])
    fd = np.array([r["fd_tip"] for r in tr])
    assert np.all(np.isfinite(lb)) and np.all(np.isfinite(fd))
    gap = np.max(np.abs(lb - fd))
    free = np.nonzero(np.maximum(lb, fd) < 0.7 * n)[0]
    sel = np.arange(len(tr) // 4, free[-1] + 1)
    assert len(sel) >= 4
    vlb = np.polyfit(steps[sel], lb[sel], 1)[0]
    vfd = np.polyfit(steps[sel], fd[sel], 1)[0]
    print("%s: max tip gap %.3f dx; free-growth velocity LB %.5f FD %.5f nodes/step (%.2f %%, "
          "%d records)" % (name, gap, vlb, vfd, 100 * (vlb / vfd - 1), len(sel)))
    assert gap <= 1.0
    assert abs(vlb - vfd) / abs(vfd) < 0.04
    assert max(abs(r["lb_solid"] - r["fd_solid"]) for r in tr) < 0.02


def _fd_anisotropy(stencil, n=150):
    name = "fd_anisotropy_%d.json" % stencil if n == 150 else "fd_anisotropy_%d_n%d.json" % (stencil, n)
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip("FD%d grid-anisotropy run (%d^3) not generated" % (stencil, n))
    with open(path) as fh:
        return json.load(fh)


def _fd_anisotropy_script():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_fd_anisotropy",
                                                  os.path.join(GOLDEN, "make_fd_anisotropy.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("stencil,n", [(6, 150), (18, 150)])
def test_fd_anisotropy_run_start_reproduces(stencil, n):
    """The stored FD6/FD18 isotropic-growth runs are what the current FD
    oracle computes: the sums of phi and theta after their first 100 steps."""
    g = _fd_anisotropy(stencil, n)
    mod = _fd_anisotropy_script()
    assert g["dt"] == mod.DT[stencil] and g["n"] == n
    s_phi, s_th = mod.check_sums(stencil, n)
    assert abs(s_phi - g["check_sum_phi"]) <= 1e-12 * abs(g["check_sum_phi"])
    assert abs(s_th - g["check_sum_theta"]) <= 1e-12 * abs(g["check_sum_theta"])


def test_fd6_explicit_step_diverges_at_the_lb_time_step():
    """The FD6 checkerboard mode grows by 1 - (12 W0^2/dx^2 + 2) dt/tau0 per
    explicit step about phi = -1: -1.1 at dt = 0.15 tau0 (divergence) and
    -0.4 at 0.1 tau0.  A small uniform liquid with a checkerboard ripple
    shows both (mirror walls lower the largest eigenvalue of the 8^3 box to
    3 * 2(1 + cos(pi/8)) = 11.5, so the factor there is -1.03 at 0.15)."""
    from oracle import FDOracle
    n = 8
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ripple = 1e-6 * (-1.0) ** (x + y + z)
    for dt, grows in ((0.15, True), (0.1, False)):
        o = FDOracle(n, n, n, lam=10.0, Mcinf=0.0, D=0.7, kappa=0.7, eps=0.0, stencil=6)
        o.set(-1.0 + ripple, np.zeros((n, n, n)), np.full((n, n, n), -0.2))
        o.step(dt, 200)
        amp = np.max(np.abs(o.fields()[0] + 1.0))
        assert (amp > 1e-5) == grows, (dt, amp)


def test_fd18_grid_is_less_anisotropic_than_fd6():
    """Sec. 4.1's FD comparison: the isotropic-growth A_g of FD6 well above
    that of FD18 (the paper: 4.365 % and 0.575 %; its undercooling is not
    printed, so the values themselves are parity unpinned).  150^3 octant,
    each stencil at its stable time step."""
    g6, g18 = _fd_anisotropy(6), _fd_anisotropy(18)
    print("A_g FD6 %.3f %%, FD18 %.3f %%" % (g6["A_g_percent"], g18["A_g_percent"]))
    assert g6["A_g_percent"] > 1.0 and g18["A_g_percent"] < 0.5


def test_fp32_rounding_evidence():
    """The stored single-precision rounding errors (the oracle's algorithm
    built in float against the FP64 oracle, tests/golden/fp32_rounding.json)
    are what the current oracles compute: the 32^3 D3Q15 ensemble domain
    after 50 steps is recomputed.  The float build does round in single
    precision (its error is far above FP64 rounding and below 1e-4), and on
    the fastest-growing cases it exceeds 1e-5 after 200 steps, which is why
    the GPU's FP32 parity there is bounded by it."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_fp32_rounding",
                                                  os.path.join(GOLDEN, "make_fp32_rounding.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with open(os.path.join(GOLDEN, "fp32_rounding.json")) as fh:
        g = json.load(fh)["cases"]
    pb = [p for p in mod.cases() if p.name == "ens-07"][0]
    got = mod.rounding_error(pb, (50,))["50"]
    assert got == g["ens-07"]["max_abs_phi_U_theta"]["50"]
    assert all(1e-9 < e < 1e-4 for e in got)
    assert g["interior"]["max_abs_phi_U_theta"]["200"][0] > 1e-5
    assert g["ens-62"]["max_abs_phi_U_theta"]["200"][0] > 1e-5
