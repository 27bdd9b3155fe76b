"""Full-size workloads on the GPU against the FP64 oracle.

Small cases are compared element by element with a live oracle run.  At full
size the oracle's reduction traces (tip position, solid fraction, solute
mass, enthalpy every R steps), written by tests/golden/make_traces.py, are
the expected values; the GPU runs in the launch configuration the benchmark
times (the library default).
"""
import json
import os

import numpy as np
import pytest

from paper_1602_07483_amd import lbpf
from paper_1602_07483_amd.inputs import (sphere_field, workload_thermal2d, workload_octant, workload_centred,
                                         workload_ensemble, workload_multiseed)
from tests.pairs import make_oracle, make_gpu, maxabs, fp32_bound

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    path = os.path.join(GOLDEN, "trace_%s.json" % name)
    if not os.path.exists(path):
        pytest.skip("oracle trace %s not generated (tests/golden/make_traces.py %s)" % (path, name))
    with open(path) as fh:
        return json.load(fh)


def run_trace(pb, storage):
    s = make_gpu(pb, storage)
    s.step(pb.steps)
    hist = s.history()
    st, red = s.read_status()
    s.close()
    assert st == lbpf.LBPF_OK, red
    return hist


def velocities(steps, tips, every):
    return np.diff(np.asarray(tips)) / float(every)


def free_growth(tips, reach):
    """Intervals whose tip stays below 90 % of the distance to the far wall.
    Once the crystal touches the wall the outermost phi = 0 crossing jumps
    between rows on field differences far below the tolerances, so the tip
    velocity there says nothing about parity."""
    t = np.asarray(tips)
    inside = t < 0.9 * reach
    return inside[:-1] & inside[1:]


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_quasi2d_slab_matches_oracle(storage, tol):
    """nz = 1 with mirror z-walls (the D2Q9 reduction of D3Q19): fields after
    300 steps of the 2D thermal dendrite parameters."""
    pb = workload_thermal2d(n=40, steps=300)
    s = make_gpu(pb, storage)
    s.step(300)
    phi, U, th, _ = s.read(reductions=False)
    o = make_oracle(pb)
    o.step(300)
    ophi, oU, oth = o.fields()
    for a, b in ((phi, ophi), (U, oU), (th, oth)):
        assert maxabs(a, b) <= tol


def test_thermal2d_tip_velocity_matches_oracle():
    """Sec. 4.1, anisotropic thermal dendrite, Delta = 0.55: FP32 GPU run of
    37 500 steps (T = 300) against the oracle's trace: tip positions within
    0.05 node and the tip velocity within 1 % past the initial transient.
    The paper's values at this resolution are printed beside it."""
    g = golden("thermal2d")
    pb = workload_thermal2d()
    hist = run_trace(pb, "f32")
    steps = [h["step"] for h in hist]
    assert steps == [r["step"] for r in g["trace"]]
    tg = [h["tip"][0] for h in hist]
    to = [r["tip"][0] for r in g["trace"]]
    assert np.max(np.abs(np.asarray(tg) - np.asarray(to))) < 0.05
    vg = velocities(steps, tg, pb.reduce_every)
    vo = velocities(steps, to, pb.reduce_every)
    late = slice(len(vo) // 3, None)          # past the initial transient
    rel = np.abs(vg[late] - vo[late]) / np.abs(vo[late])
    print("thermal2d tip velocity rel. error (FP32 vs oracle): max %.3e" % rel.max())
    assert rel.max() < 0.01
    d0 = 0.8839 / pb.lam                       # a1 W0 / lambda
    vp = vg[-1] * pb.dx / pb.dt * d0 / pb.kappa
    print("thermal2d V_p(T=300): GPU %.5f (paper: LB 0.01735, FD/MC 0.01667, GF 0.0170)" % vp)


def _thermal2d_vp(dx, box=200.0, T=300.0, **over):
    """V_p at time T of the Sec. 4.1 thermal dendrite refined to dx/W0
    (dt proportional to dx^2, seed radius 4 W0) in a box of `box` W0,
    FP32, theta alone."""
    pb = workload_thermal2d(n=int(round(box / dx)), dx=dx)
    pb.steps = int(round(T / pb.dt))
    pb.reduce_every = int(round(4.0 / pb.dt))
    s = make_gpu(pb, "f32", skip_U=1, **over)
    s.step(pb.steps)
    hist = s.history()
    st, red = s.read_status()
    s.close()
    assert st == lbpf.LBPF_OK, red
    tips = np.array([h["tip"][0] for h in hist])
    steps = np.array([h["step"] for h in hist], dtype=float)
    v = np.diff(tips)[-1] / np.diff(steps)[-1] * pb.dx / pb.dt
    return v * (0.8839 / pb.lam) / pb.kappa


def test_thermal2d_refinement_converges_to_the_green_function_value():
    """The same dendrite at dx/W0 = 0.4, 0.3, 0.2 (dt proportional to dx^2,
    T = 300, the 200 W0 quadrant of the paper): V_p rises by equal steps for
    equal steps of dx, i.e. the scheme converges at first order, and the
    first-order extrapolation to dx = 0 lies within 1 % of the
    Green's-function value 0.0170 that Sec. 4.1 quotes.  At dx/W0 = 0.4 it
    equals the oracle's stored value (tests/golden/trace_thermal2d.json)
    within 0.1 %."""
    v = {h: _thermal2d_vp(h) for h in (0.4, 0.3, 0.2)}
    d1, d2 = v[0.3] - v[0.4], v[0.2] - v[0.3]
    v0 = 2.0 * v[0.2] - v[0.4]
    print("V_p(T=300) at dx/W0 = 0.4, 0.3, 0.2: %.5f %.5f %.5f; extrapolated %.5f (%+.2f %% from 0.0170)"
          % (v[0.4], v[0.3], v[0.2], v0, 100 * (v0 / 0.0170 - 1)))
    assert d1 > 0 and d2 > 0 and 0.6 < d1 / d2 < 1.6
    assert abs(v0 - 0.0170) / 0.0170 < 0.01
    g = golden("thermal2d")
    pb = workload_thermal2d()
    to = [r["tip"][0] for r in g["trace"]]
    vo = (to[-1] - to[-2]) / pb.reduce_every * pb.dx / pb.dt * (0.8839 / pb.lam) / pb.kappa
    assert abs(v[0.4] - vo) / vo < 1e-3


def test_thermal2d_steady_velocity_does_not_depend_on_the_initial_width():
    """Reading R11 sets the initial tanh profile's width to sqrt(2) W0 (the
    printed width is garbled).  With the initial profile half as wide,
    V_p(T = 300) at dx/W0 = 0.4 is that of the R11 run within 0.3 %
    (observed equal); twice as wide, the profile is still relaxing and V_p
    is lower, within 1 % (observed -0.7 %).  No width moves V_p up towards
    the paper's LB value (5.9 % above), so the initial width is not behind
    that gap."""
    def vp(width):
        pb = workload_thermal2d()
        s = lbpf.solver_for(pb, storage="f32", skip_U=1)
        _, U, th = pb.initial_fields()
        s.set_fields(sphere_field(pb.shape, pb.centres, pb.radius, W0=width, dx=pb.dx), U, th)
        s.step(pb.steps)
        hist = s.history()
        st, red = s.read_status()
        s.close()
        assert st == lbpf.LBPF_OK, red
        tips = np.array([h["tip"][0] for h in hist])
        steps = np.array([h["step"] for h in hist], dtype=float)
        v = np.diff(tips)[-1] / np.diff(steps)[-1] * pb.dx / pb.dt
        return v * (0.8839 / pb.lam) / pb.kappa
    v = {w: vp(w) for w in (0.5, 1.0, 2.0)}
    print("V_p(T=300) with the initial width x0.5, x1, x2: %.5f %.5f %.5f" % (v[0.5], v[1.0], v[2.0]))
    assert abs(v[0.5] - v[1.0]) / v[1.0] < 3e-3
    assert abs(v[2.0] - v[1.0]) / v[1.0] < 1e-2
    assert max(v.values()) < 1.003 * v[1.0]


def test_thermal2d_tip_velocity_does_not_depend_on_the_tip_estimator():
    """Reading R16 places the tip at the linearly interpolated phi = 0
    crossing.  A quadratic crossing through three nodes around it moves each
    position by a near-constant amount while the tip advances steadily, so
    the velocity between T = 296 and T = 300 (dx/W0 = 0.4) must agree within
    0.2 % whichever is used, and the linear one equals the library's reduced
    tip velocity."""
    pb = workload_thermal2d()
    s = lbpf.solver_for(pb, storage="f32", skip_U=1)
    s.set_fields(*pb.initial_fields())
    every = pb.reduce_every
    s.step(pb.steps - every)
    rows = [s.read()[0][0, 0, :]]
    s.step(every)
    phi, _, _, red = s.read()
    rows.append(phi[0, 0, :])
    hist = s.history()
    s.close()

    def tips(row):
        i = int(np.nonzero((row[:-1] > 0) & (row[1:] <= 0))[0].max())
        lin = i + row[i] / (row[i] - row[i + 1])
        a, b, c = row[i - 1], row[i], row[i + 1]   # parabola through i-1, i, i+1 (t = x - i)
        qa, qb, qc = 0.5 * (a + c) - b, 0.5 * (c - a), b
        r = np.roots([qa, qb, qc])
        quad = i + float(np.real(r[(np.isreal(r)) & (np.real(r) >= 0) & (np.real(r) <= 1)][0]))
        return lin, quad

    (l0, q0), (l1, q1) = tips(rows[0]), tips(rows[1])
    scale = pb.dx / pb.dt * (0.8839 / pb.lam) / pb.kappa / every
    v_lin, v_quad = (l1 - l0) * scale, (q1 - q0) * scale
    v_red = (hist[-1]["tip"][0] - hist[-2]["tip"][0]) * scale
    print("V_p(T=300): linear %.5f, quadratic %.5f, reduction %.5f" % (v_lin, v_quad, v_red))
    assert abs(v_quad - v_lin) / v_lin < 2e-3
    assert abs(v_red - v_lin) / v_lin < 1e-6


def test_thermal2d_tip_velocity_paper_lattices():
    """Sec. 4.1's own lattice pair: the phase field on D2Q9 and theta on
    D2Q5, here a one-node slab with phi on D3Q19 (D2Q9 after the mirror
    reduction) and theta on D3Q7 (a D2Q5), pure substance (theta alone),
    FP32, T = 300: V_p within 0.5 % of the all-D2Q9 value of the oracle's
    stored run, so the theta lattice does not move the tip velocity."""
    pb = workload_thermal2d()
    s = make_gpu(pb, "f32", skip_U=1, lattice_ut=7)
    s.step(pb.steps)
    hist = s.history()
    st, red = s.read_status()
    s.close()
    assert st == lbpf.LBPF_OK, red
    tips = [h["tip"][0] for h in hist]
    v = velocities(None, tips, pb.reduce_every)
    d0 = 0.8839 / pb.lam
    vp = v[-1] * pb.dx / pb.dt * d0 / pb.kappa
    to = [r["tip"][0] for r in golden("thermal2d")["trace"]]
    vo = (to[-1] - to[-2]) / pb.reduce_every * pb.dx / pb.dt * d0 / pb.kappa
    print("thermal2d D2Q9 phi + D2Q5 theta: V_p(T=300) %.5f, all-D2Q9 oracle %.5f" % (vp, vo))
    assert abs(vp - vo) / vo < 0.005


def test_octant128_tip_velocity_matches_oracle():
    """128^3 octant dendrite, 5000 FP32 steps, reductions every 100 steps:
    tip velocity within 1 %, solid fraction and solute mass against the
    oracle's trace."""
    g = golden("octant128")
    pb = workload_octant(128, 5000)
    hist = run_trace(pb, "f32")
    assert [h["step"] for h in hist] == [r["step"] for r in g["trace"]]
    for h, r in zip(hist, g["trace"]):
        assert abs(h["solid_fraction"] - r["solid_fraction"]) < 1e-5
        assert abs(h["solute_mass"] - r["solute_mass"]) < 1e-5 * abs(r["solute_mass"])
        assert abs(h["tip"][0] - r["tip"][0]) < 0.05
    vg = velocities(None, [h["tip"][0] for h in hist], pb.reduce_every)
    vo = velocities(None, [r["tip"][0] for r in g["trace"]], pb.reduce_every)
    ok = free_growth([r["tip"][0] for r in g["trace"]], pb.nx) & (np.abs(vo) > 1e-3)
    rel = np.abs(vg[ok] - vo[ok]) / np.abs(vo[ok])
    print("octant128 tip velocity rel. error FP32: %.3e over %d intervals" % (rel.max(), ok.sum()))
    assert ok.sum() >= 5 and rel.max() < 0.01


@pytest.mark.parametrize("storage,bound", [("f32", 0.01), ("f16", 0.01), ("bf16", 0.01)])
def test_centred256_tip_velocity_matches_oracle(storage, bound):
    """256^3 centred seed, 10 000 steps, FP64 reductions every 100 steps,
    against the oracle's trace of the equivalent octant (mirror walls through
    the seed centre): tip velocity within 1 % (FP32 and mixed storage),
    solid fraction, and solute-mass drift."""
    g = golden("centred256")
    pb = workload_centred(256, 10000)
    hist = run_trace(pb, storage)
    tr = g["trace"]
    assert [h["step"] for h in hist] == [r["step"] for r in tr]
    vg = velocities(None, [h["tip"][0] for h in hist], pb.reduce_every)
    vo = velocities(None, [r["tip"][0] for r in tr], pb.reduce_every)
    ok = free_growth([r["tip"][0] for r in tr], pb.nx // 2) & (np.abs(vo) > 1e-3)
    rel = np.abs(vg[ok] - vo[ok]) / np.abs(vo[ok])
    fs = max(abs(h["solid_fraction"] - r["solid_fraction"]) for h, r in zip(hist, tr))
    m0 = 8.0 * tr[0]["solute_mass"]
    drift_g = (hist[-1]["solute_mass"] - hist[0]["solute_mass"]) / abs(hist[0]["solute_mass"])
    drift_o = (8.0 * tr[-1]["solute_mass"] - m0) / abs(m0)
    print("centred256 %s: tip velocity rel. error %.3e over %d intervals; |d solid fraction| %.2e; "
          "mass drift GPU %.3e oracle %.3e" % (storage, rel.max(), ok.sum(), fs, drift_g, drift_o))
    assert ok.sum() >= 5 and rel.max() < bound
    # solid fraction over the whole run; mixed storage reported with loose bounds
    assert fs < {"f32": 1e-5, "f16": 2e-3, "bf16": 1e-2}[storage]


def test_ensemble_health_and_sampled_parity():
    """The 64-domain ensemble, batched in mixed FP16 storage with graph
    replay: every domain healthy after 2000 steps, and the smallest and
    largest domain of each lattice against the oracle after 200 steps
    (FP32 batch, element by element).

    Tolerance per domain and field: 1e-5, or what the oracle's own
    algorithm rounded to float reaches on that domain after 200 steps where
    that is larger (tests/golden/fp32_rounding.json, written by
    tests/golden/make_fp32_rounding.py).  The largest D3Q19 domain (95^3,
    Delta = 0.52, eps = 0.061) grows fastest; the growing tips amplify the
    rounding of any FP32 state (one rounding of phi, U, theta per node and
    step) about 1.5x every 25 steps after step 75, and the float algorithm
    reaches 1.9e-5 on phi there, the GPU about 1.2e-5."""
    probs = workload_ensemble()
    b = lbpf.Batch([lbpf.problem_kwargs(p) for p in probs], storage="f16")
    for d, p in zip(b.domains, probs):
        d.set_fields(*p.initial_fields())
    b.set_graph(50)
    b.step(2000)
    reds = [d.read_status()[1] for d in b.domains]
    b.close()
    # all finite; the health bound |phi| <= 1 + 1e-3 wherever the cubic
    # stiffness 1 - 15 eps is positive (eps > 1/15 is ill-posed: reported)
    assert all(r["nonfinite"] == 0 for r in reds)
    for p, r in zip(probs, reds):
        peak = max(-r["phi_min"], r["phi_max"])
        if p.eps > 1.0 / 15.0:
            print("%s eps %.4f > 1/15: max|phi| %.4f" % (p.name, p.eps, peak))
        else:
            assert peak <= 1.0 + 1e-3, (p.name, p.lattice, p.eps, r)
    half = len(probs) // 2
    picks = []
    for part in (probs[:half], probs[half:]):
        order = sorted(part, key=lambda p: p.nodes)
        picks += [order[0], order[-1]]
    b = lbpf.Batch([lbpf.problem_kwargs(p) for p in picks], storage="f32")
    for d, p in zip(b.domains, picks):
        d.set_fields(*p.initial_fields())
    b.step(200)
    for d, p in zip(b.domains, picks):
        phi, U, th, _ = d.read(reductions=False)
        o = make_oracle(p)
        o.step(200)
        ophi, oU, oth = o.fields()
        print("%s (Q%d, %d^3): max|dphi| %.2e max|dU| %.2e" % (p.name, p.lattice, p.nx,
                                                              maxabs(phi, ophi), maxabs(U, oU)))
        for f, (got, want) in enumerate(((phi, ophi), (U, oU), (th, oth))):
            assert maxabs(got, want) <= fp32_bound(p.name, f), (p.name, f, maxabs(got, want))
    b.close()


def _subbox_oracle(pb, fields0, node, r, steps):
    """Oracle values at `node` after `steps` steps, computed on the cube of
    half-width r around it cut out of the full initial fields.  One step
    reaches at most 4 nodes (pull link + stencils of phi^n and phi^{n+1}) and
    the equilibrium start one more, so r >= 4 steps + 2 keeps the cut faces
    out of the node's domain of dependence."""
    from oracle import Oracle
    x, y, z = node
    sl = (slice(z - r, z + r + 1), slice(y - r, y + r + 1), slice(x - r, x + r + 1))
    kw = pb.model_kwargs()
    kw["walls"] = (0,) * 6
    o = Oracle(2 * r + 1, 2 * r + 1, 2 * r + 1, **kw)
    o.init(*(np.ascontiguousarray(f[sl]) for f in fields0))
    o.step(steps)
    vals = [f[r, r, r] for f in o.fields()]
    o.close()
    return vals


@pytest.mark.parametrize("storage,aniso,tol", [("f32", 0, 1e-5), ("f16", 0, 5e-3),
                                               ("f32", 1, 1e-5), ("bf16", 1, 5e-2)])
def test_multiseed512_sampled_parity(storage, aniso, tol):
    """512^3, 8 nuclei, cubic or K41/K61 anisotropy, FP32 or mixed storage
    (at this size every field exceeds 4 GiB of populations, so the kernels
    use 64-bit addressing): after 8 steps, phi, U and theta at 24 nodes on
    and around the nuclei against the oracle run on a sub-cube per node."""
    steps, r = 8, 35
    pb = workload_multiseed(512, aniso=aniso)
    fields0 = pb.initial_fields()
    s = make_gpu(pb, storage)
    s.step(steps)
    phi, U, th, _ = s.read(reductions=False)
    s.close()
    nodes = []
    for c in pb.centres:
        b = [int(round(v)) for v in c]
        sx, sy, sz = (1 if v < 256 else -1 for v in b)         # offsets point inwards
        nodes.append((b[0] + 6 * sx, b[1], b[2]))              # on the interface
        nodes.append((b[0], b[1] + 5 * sy, b[2] + 3 * sz))     # inside, off axis
        nodes.append((b[0] + 4 * sx, b[1] + 4 * sy, b[2] + 4 * sz))   # near the <111> front
    worst = 0.0
    for node in nodes:
        assert all(r <= v < 512 - r for v in node), node
        want = _subbox_oracle(pb, fields0, node, r, steps)
        x, y, z = node
        got = (phi[z, y, x], U[z, y, x], th[z, y, x])
        err = max(abs(a - b) for a, b in zip(got, want))
        worst = max(worst, err)
    print("multiseed512 %s aniso %d: max error at %d sampled nodes %.3e" % (storage, aniso, len(nodes), worst))
    assert worst <= tol


@pytest.mark.parametrize("storage,bound", [("f32", 1e-7), ("f16", 1e-5)])
def test_multiseed512_enthalpy_conserved(storage, bound):
    """Sum of (theta - phi/2) is an exact invariant of the scheme with
    no-flux walls (the theta source is half the phi increment); at 512^3 the
    FP64 reductions of the FP32/mixed run must keep it to the stated bound
    per node over 200 steps."""
    pb = workload_multiseed(512, aniso=0)
    pb.reduce_every = 50
    s = make_gpu(pb, storage)
    _, red0 = s.read_status()
    s.step(200)
    hist = s.history()
    s.close()
    h0 = red0["enthalpy"]
    drift = max(abs(h["enthalpy"] - h0) for h in hist) / pb.nodes
    print("multiseed512 %s: enthalpy drift per node %.3e; solid fraction %.6f -> %.6f"
          % (storage, drift, red0["solid_fraction"], hist[-1]["solid_fraction"]))
    assert drift <= bound


def _first_crossing(prof):
    i = np.nonzero((prof[:-1] > 0) & (prof[1:] <= 0))[0]
    assert len(i), "no phi = 0 crossing"
    i = i[0]
    return i + prof[i] / (prof[i] - prof[i + 1])


def test_grid_anisotropy_of_isotropic_growth():
    """Sec. 4.1, isotropic case (eps = 0): a sphere of radius 8 grows for
    10^4 steps at dx = W0, dt = 0.15 tau0, kappa dt/dx^2 = 0.105, lambda = 10
    (pure substance), on a 150^3 octant (the 300^3 domain about its centre).
    The grid anisotropy A_g = |R100 - R110| / (R100 + R110) is large on D3Q7
    and small on D3Q15 and D3Q19, as the paper reports (3.1 %, 0.07 %,
    0.12 %).  The paper does not print the undercooling, so Delta = 0.2 is
    chosen here and the exact values are parity unpinned."""
    from paper_1602_07483_amd.inputs import Problem, NOFLUX, SYMMETRY
    n = 150
    walls = (SYMMETRY, NOFLUX, SYMMETRY, NOFLUX, SYMMETRY, NOFLUX)
    ag, radii = {}, {}
    # (phi lattice, theta lattice); the last runs phi on D3Q19 and theta on
    # D3Q7, as Sec. 4.1 runs D2Q9 with D2Q5 in 2D: reported only
    for lat, lat_t in ((7, 7), (15, 15), (19, 19), (19, 7)):
        pb = Problem("isotropic", n, n, n, lat, walls, dx=1.0, dt=0.15, W0=1.0, tau0=1.0, lam=10.0,
                     Mcinf=0.0, k=0.15, D=0.7, kappa=0.7, eps=0.0, centres=[(-0.5, -0.5, -0.5)],
                     radius=8.0, U0=0.0, theta0=-0.2)
        s = make_gpu(pb, "f32", skip_U=1, lattice_ut=lat_t)      # pure substance: theta alone
        s.step(10000)
        phi, _, _, red = s.read(check=False)
        s.close()
        assert red["nonfinite"] == 0 and max(-red["phi_min"], red["phi_max"]) < 1.01
        r100 = _first_crossing(phi[0, 0, :]) + 0.5                      # from the mirror point
        r110 = (_first_crossing(np.array([phi[0, i, i] for i in range(n)])) + 0.5) * np.sqrt(2.0)
        assert 20.0 < r100 < 0.7 * n
        key = lat if lat == lat_t else (lat, lat_t)
        radii[key] = (r100, r110)
        ag[key] = abs(r100 - r110) / (r100 + r110) * 100.0
        print("phi D3Q%d theta D3Q%d: R100 %.3f R110 %.3f A_g %.3f %%" % (lat, lat_t, r100, r110, ag[key]))
    assert ag[7] > 1.0
    assert ag[15] < 0.5 and ag[19] < 0.5
    # the FD oracle's FD6 and FD18 runs of the same setup (written by
    # tests/golden/make_fd_anisotropy.py), which the paper sets beside its lattices
    for st in (6, 18):
        path = os.path.join(GOLDEN, "fd_anisotropy_%d.json" % st)
        if os.path.exists(path):
            with open(path) as fh:
                g = json.load(fh)
            print("FD%d (oracle): R100 %.3f R110 %.3f A_g %.3f %%" % (st, g["R100"], g["R110"], g["A_g_percent"]))
            if st == 18:
                # the paper finds the LB-D3Q19 and FD18 circles to coincide
                assert abs(radii[19][0] - g["R100"]) < 0.02 * g["R100"]
                assert abs(radii[19][1] - g["R110"]) < 0.02 * g["R110"]


def _last_crossing(prof):
    i = np.nonzero((prof[:-1] > 0) & (prof[1:] <= 0))[0]
    assert len(i), "no phi = 0 crossing"
    i = i[-1]
    return i + prof[i] / (prof[i] - prof[i + 1])


@pytest.mark.parametrize("aniso,eps,delta,steps", [(0, 0.05, 0.0, 10000), (1, 0.0, -0.02, 40000)])
def test_preferred_growth_direction_sec_4_3(aniso, eps, delta, steps):
    """Sec. 4.3 (non-standard dendrites) with the paper's parameters:
    dx = 0.01, dt = 1.5e-5, W0 = 0.0125, tau0 = 1.5625e-4, lambda = 10,
    kappa = 1, Delta = 0.25, seed R = 8 at the corner of mirror planes, pure
    substance, in a 176^3 octant (half the paper's 351 nodes of reach, so
    the runs stop before the crystal meets the far walls).  The cubic
    function with eps = 0.05 grows along [100]; the K41/K61 function with
    eps = 0, delta = -0.02 along [110], as in the paper's figure."""
    from paper_1602_07483_amd.inputs import Problem, NOFLUX, SYMMETRY
    n = 176
    walls = (SYMMETRY, NOFLUX, SYMMETRY, NOFLUX, SYMMETRY, NOFLUX)
    pb = Problem("sec4.3", n, n, n, 19, walls, dx=0.01, dt=1.5e-5, W0=0.0125, tau0=1.5625e-4,
                 lam=10.0, Mcinf=0.0, k=0.15, D=1.0, kappa=1.0, aniso=aniso, eps=eps, delta=delta,
                 centres=[(-0.5, -0.5, -0.5)], radius=8.0, U0=0.0, theta0=-0.25)
    s = make_gpu(pb, "f32", skip_U=1)          # pure substance: U does not act on phi
    s.step(steps)
    phi, _, _, red = s.read(check=False)
    s.close()
    assert red["nonfinite"] == 0
    r100 = _last_crossing(phi[0, 0, :]) + 0.5
    r110 = (_last_crossing(np.array([phi[0, i, i] for i in range(n)])) + 0.5) * np.sqrt(2.0)
    r111 = (_last_crossing(np.array([phi[i, i, i] for i in range(n)])) + 0.5) * np.sqrt(3.0)
    print("Sec. 4.3 aniso %d after %d steps: R100 %.2f R110 %.2f R111 %.2f (lattice units)"
          % (aniso, steps, r100, r110, r111))
    assert max(r100, r110, r111) < 0.95 * n
    if aniso == 0:
        assert r100 > 1.1 * r110 and r100 > 1.1 * r111
    else:
        assert r110 > 1.1 * r100 and r110 > 1.1 * r111


def _tip_along_x(phi, cx):
    """Largest phi = 0 crossing along +x over all rows (linear interpolation),
    minus cx: the tip measure of the stored LB-versus-FD traces."""
    a, b = phi[..., :-1], phi[..., 1:]
    m = (a > 0) & (b <= 0)
    if not m.any():
        return float("nan")
    x = np.arange(phi.shape[-1] - 1, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        xs = np.where(m, x + a / np.where(m, a - b, 1.0), -np.inf)
    return float(xs.max()) - cx


@pytest.mark.parametrize("storage,tol", [("f32", 0.02), ("f16", 0.2)])
def test_isothermal_alloy_benchmark_matches_oracle(storage, tol):
    """The paper's isothermal alloy benchmark (Sec. 4.2: dx/W0 = 0.4,
    dt/tau0 = 0.02, U0 = -0.55, D = 2, k = 0.15, eps = 0.03, lambda = 3.2,
    R_s = 10, theta = 0) in a 64^3 octant with skip_theta: the tip position
    every 50 steps against the FP64 oracle's isothermal run stored in
    tests/golden/trace_fd3d_iso.json (tol nodes), and the free-growth tip
    velocity within 1 %."""
    from paper_1602_07483_amd.inputs import Problem
    g = golden("fd3d_iso")
    p = dict(g["problem"])
    pb = Problem(**{k: (tuple(v) if isinstance(v, list) and k == "walls" else v) for k, v in p.items()})
    pb.centres = [tuple(c) for c in pb.centres]
    s = make_gpu(pb, storage, skip_theta=1)
    cx = pb.centres[0][0]
    gpu, ref, steps = [], [], []
    done = 0
    for rec in g["trace"]:
        s.step(rec["step"] - done)
        done = rec["step"]
        phi = s.read(reductions=False)[0]
        gpu.append(_tip_along_x(phi, cx))
        ref.append(rec["lb_tip"])
        steps.append(done)
    s.close()
    gpu, ref, steps = np.array(gpu), np.array(ref), np.array(steps, dtype=float)
    gap = np.max(np.abs(gpu - ref))
    free = np.nonzero(ref < 0.7 * pb.nx)[0]
    sel = np.arange(len(ref) // 4, free[-1] + 1)
    vg = np.polyfit(steps[sel], gpu[sel], 1)[0]
    vr = np.polyfit(steps[sel], ref[sel], 1)[0]
    print("isothermal benchmark %s: max tip gap %.4f nodes, velocity GPU %.5f oracle %.5f (%.3f %%)"
          % (storage, gap, vg, vr, 100 * (vg / vr - 1)))
    assert gap <= tol
    assert abs(vg / vr - 1) < 0.01
