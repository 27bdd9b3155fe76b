"""GPU runtime features through the C ABI: launch shapes, graph replay,
batched ensembles, checkpoint/restore, health checks and the FP64 reductions
against the oracle."""
import dataclasses

import numpy as np
import pytest

from oracle import Oracle, R_SOLID, R_MASS, R_ENTHALPY, R_TIPX, R_TIPY, R_TIPZ
from paper_1602_07483_amd import lbpf
from paper_1602_07483_amd.build import kernel_build_id
from paper_1602_07483_amd.inputs import workload_interior, Problem, workload_small, workload_octant, NOFLUX, SYMMETRY, DT
from tests.pairs import make_oracle, make_gpu, maxabs

pytestmark = pytest.mark.gpu


def ragged(lattice=19, n=(45, 23, 21), aniso=0, eps=0.05, delta=0.0, U0=-0.55, seed=3,
           walls=(SYMMETRY, NOFLUX, NOFLUX, SYMMETRY, SYMMETRY, NOFLUX)):
    nx, ny, nz = n
    return Problem("ragged", nx, ny, nz, lattice, walls, dt=DT, aniso=aniso, eps=eps, delta=delta,
                   centres=[(-0.5, ny - 0.5, -0.5)], radius=6.0, U0=U0, theta0=U0,
                   noise_amp=1e-3, noise_seed=seed)


def fields(s):
    phi, U, th, _ = s.read(reductions=False)
    return phi, U, th


@pytest.mark.parametrize("case", ["ragged", "interior"])
def test_launch_shape_does_not_change_results(case):
    """Tile shape, slab height and XCD order change speed only: bit-identical
    fields, on the ragged case (every tile touches a wall) and on the
    136x40x24 interior case (some tiles of every shape take the wall-free
    path, others the wall path)."""
    pb = ragged() if case == "ragged" else workload_interior()
    ref = None
    for launch in [(32, 8, 6, 1), (64, 2, 8, 1), (32, 4, 2, 0), (64, 4, 16, 1), (32, 16, 4, 1), (32, 8, 1, 0)]:
        s = make_gpu(pb, "f32")
        s.set_launch(*launch)
        s.step(40)
        out = fields(s)
        s.close()
        if ref is None:
            ref = out
        else:
            for a, b in zip(ref, out):
                assert np.array_equal(a, b), launch
    # the two kernels on different launches
    for phi_l, ut_l in [((64, 4, 6, 1), (32, 8, 2, 0)), ((32, 16, 3, 0), (64, 2, 5, 1))]:
        s = make_gpu(pb, "f32")
        s.set_kernel_launch(0, *phi_l)
        s.set_kernel_launch(1, *ut_l)
        assert s.launches() == {"k_phi": phi_l, "k_ut": ut_l}
        s.step(40)
        out = fields(s)
        s.close()
        for a, b in zip(ref, out):
            assert np.array_equal(a, b), (phi_l, ut_l)


def test_graph_replay_equals_plain_launches():
    """Replays of a captured graph, with reads and plain steps in between,
    match plain launches bit for bit after every replay."""
    pb = ragged(lattice=15, n=(40, 33, 17))
    plain = make_gpu(pb, "f32")
    graph = make_gpu(pb, "f32")
    graph.set_graph(4)
    for chunk in (3, 8, 4, 1, 12, 4):
        plain.step(chunk)
        graph.step(chunk)
        a, b = fields(plain), fields(graph)
        for x, y in zip(a, b):
            assert np.array_equal(x, y), chunk
    graph.set_launch(32, 4, 4, 1)   # new shape: the graph is captured again
    plain.set_launch(32, 4, 4, 1)
    graph.step(8)
    plain.step(8)
    for x, y in zip(fields(plain), fields(graph)):
        assert np.array_equal(x, y)


def _batch_problems():
    return [ragged(15, (33, 21, 19), eps=0.03, U0=-0.5, seed=11),
            ragged(19, (40, 35, 24), eps=0.06, U0=-0.6, seed=12),
            ragged(15, (64, 8, 9), eps=0.02, U0=-0.45, seed=13, walls=(NOFLUX,) * 6),
            ragged(19, (17, 40, 33), aniso=1, eps=0.0, delta=-0.02, seed=14),
            ragged(19, (29, 29, 29), eps=0.07, U0=-0.65, seed=15, walls=(SYMMETRY,) * 6),
            dataclasses.replace(ragged(7, (37, 21, 19), eps=0.04, U0=-0.5, seed=16), dt=0.11)]


@pytest.mark.parametrize("graph_steps", [0, 6])
def test_batch_matches_domains_stepped_alone(graph_steps):
    """Each domain of a mixed D3Q7/D3Q15/D3Q19 batch against the same domain
    stepped alone.  The batch kernels are compiled separately (coefficients
    come from a descriptor), so contraction into FMAs may differ: after 25
    steps the fields agree to a few ulp of values of order one."""
    probs = _batch_problems()
    b = lbpf.Batch([lbpf.problem_kwargs(p) for p in probs], storage="f32")
    for d, p in zip(b.domains, probs):
        d.set_fields(*p.initial_fields())
    b.set_graph(graph_steps)
    b.step(7)
    b.step(18)
    got = [fields(d) for d in b.domains]
    for p, g in zip(probs, got):
        s = make_gpu(p, "f32")
        s.step(25)
        for x, y in zip(fields(s), g):
            assert maxabs(x, y) <= 1e-6, p
        s.close()
    b.close()


def test_batch_graph_and_chunking_are_bit_exact():
    """Within the batch, graph replay and step chunking change nothing."""
    probs = _batch_problems()
    outs = []
    for graph_steps, chunks in ((0, (25,)), (6, (7, 18)), (4, (1, 3, 21))):
        b = lbpf.Batch([lbpf.problem_kwargs(p) for p in probs], storage="f32")
        for d, p in zip(b.domains, probs):
            d.set_fields(*p.initial_fields())
        b.set_graph(graph_steps)
        for c in chunks:
            b.step(c)
        outs.append([fields(d) for d in b.domains])
        b.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_batch_launch_and_autotune(storage):
    """Batch launches per kernel (tile shape and z slab for k_phi and k_ut
    apart) and the batch autotuner.  Another tile shape is another
    instantiation of the batch kernels, whose constants come from a
    descriptor, so the compiler may contract multiply-adds differently:
    after 20 steps the fields agree with the default launch to a few ulp.
    The tuner restores every domain's state: a batch tuned after 6 steps and
    stepped 14 more equals, bit for bit, one set to the tuned launches by
    hand at the same point (graph replay captured again after each change)."""
    probs = _batch_problems()

    def run(setup):
        b = lbpf.Batch([lbpf.problem_kwargs(p) for p in probs], storage=storage)
        for d, p in zip(b.domains, probs):
            d.set_fields(*p.initial_fields())
        b.set_graph(4)
        b.step(6)
        setup(b)
        b.step(14)
        out = [fields(d) for d in b.domains]
        launches = (b.get_launch(0), b.get_launch(1))
        b.close()
        return out, launches

    ref, l0 = run(lambda b: None)
    assert l0[0][:2] == (32, 8) and l0[1][:2] == (32, 8)

    def mixed(b):
        b.set_launch(0, 32, 4, 2)
        b.set_launch(1, 64, 4, 12)

    got, launches = run(mixed)
    assert launches == ((32, 4, 2), (64, 4, 12))
    tol = 1e-6 if storage == "f32" else 1e-3
    for a, g in zip(ref, got):
        for x, y in zip(a, g):
            assert maxabs(x, y) <= tol

    def tuned(b):
        launches, best = b.autotune(1)
        assert best > 0 and set(launches) == {"k_phi", "k_ut"}

    got_t, lt = run(tuned)
    print(storage, "tuned launches", lt)

    def by_hand(b):
        b.set_launch(0, *lt[0])
        b.set_launch(1, *lt[1])

    got_h, lh = run(by_hand)
    assert lh == lt
    for a, g in zip(got_h, got_t):
        for x, y in zip(a, g):
            assert np.array_equal(x, y)


def test_batch_fp64_matches_oracle():
    probs = _batch_problems()[:3] + _batch_problems()[5:]   # D3Q15, D3Q19, D3Q7
    b = lbpf.Batch([lbpf.problem_kwargs(p) for p in probs], storage="f64")
    for d, p in zip(b.domains, probs):
        d.set_fields(*p.initial_fields())
    b.step(30)
    for d, p in zip(b.domains, probs):
        o = make_oracle(p)
        o.step(30)
        for x, y in zip(fields(d), o.fields()):
            assert maxabs(x, y) <= 1e-12
    b.close()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_checkpoint_restore_is_bit_exact(storage):
    """Fields plus raw stored populations restore the state exactly."""
    pb = ragged()
    s = make_gpu(pb, storage)
    s.step(20)
    phi, U, th = fields(s)
    pops = [s.read_populations(f) for f in range(3)]
    s.step(15)
    want = fields(s)
    r = lbpf.solver_for(pb, storage=storage)
    r.set_fields(phi, U, th)
    for f in range(3):
        r.write_populations(f, pops[f])
    r.step(15)
    for x, y in zip(want, fields(r)):
        assert np.array_equal(x, y)


def test_health_check_reports_unstable_state():
    pb = ragged()
    phi, U, th = pb.initial_fields()
    U = U.copy()
    U[3, 4, 5] = np.nan
    pb.reduce_every = 2
    s = lbpf.solver_for(pb, storage="f32")
    s.set_fields(phi, U, th)
    s.step(2)
    assert s.sync(check=False) == lbpf.LBPF_EUNSTABLE
    st, red = s.read_status()
    assert st == lbpf.LBPF_EUNSTABLE and red["nonfinite"] > 0
    phi2 = pb.initial_fields()[0].copy()
    phi2[0, 0, 0] = 5.0
    s2 = make_gpu(pb, "f32")
    s2.set_fields(phi2, *pb.initial_fields()[1:])
    st, red = s2.read_status()
    assert st == lbpf.LBPF_EUNSTABLE and red["phi_max"] == 5.0
    healthy = make_gpu(pb, "f32")
    healthy.step(5)
    assert healthy.read_status()[0] == lbpf.LBPF_OK


def test_reductions_and_tip_velocity_match_oracle():
    """FP64 reductions of the FP32 run against the oracle's: solid fraction,
    solute mass, enthalpy, tip positions; tip velocity within 1 %."""
    pb = workload_octant(n=48, steps=400)
    pb.reduce_every = 50
    s = make_gpu(pb, "f32")
    s.step(400)
    hist = s.history()
    assert [h["step"] for h in hist] == list(range(50, 401, 50))
    o = make_oracle(pb)
    tips_g, tips_o = [], []
    for h in hist:
        o.step(50)
        r = o.reduce(pb.centre())
        assert abs(h["solid_fraction"] - r[R_SOLID]) < 1e-6
        assert abs(h["solute_mass"] - r[R_MASS]) < 1e-6 * abs(r[R_MASS])
        assert abs(h["enthalpy"] - r[R_ENTHALPY]) < 1e-6 * pb.nodes
        tips_g.append(h["tip"][0])
        tips_o.append(r[R_TIPX])
        for a, key in enumerate((R_TIPX, R_TIPY, R_TIPZ)):
            assert abs(h["tip"][a] - r[key]) < 1e-3
    vg = np.diff(tips_g) / 50.0
    vo = np.diff(tips_o) / 50.0
    ok = np.abs(vo) > 1e-3
    assert ok.sum() >= 3
    rel = np.abs(vg[ok] - vo[ok]) / np.abs(vo[ok])
    print("tip velocity rel. error FP32:", rel.max())
    assert rel.max() < 0.01
    # the library's own tip velocity: the same difference in physical units
    assert all(np.isnan(hist[0]["tip_vel"]))
    for h0, h1 in zip(hist[:-1], hist[1:]):
        for a in range(3):
            expect = (h1["tip"][a] - h0["tip"][a]) * pb.dx / ((h1["step"] - h0["step"]) * pb.dt)
            assert h1["tip_vel"][a] == pytest.approx(expect, rel=1e-12, abs=1e-15)
    s.step(25)                                   # lbpf_read: against the last record (step 400)
    red = s.read()[3]
    assert red["tip_vel"][0] == pytest.approx((red["tip"][0] - hist[-1]["tip"][0]) * pb.dx / (25 * pb.dt),
                                              rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("storage,bound", [("f16", 0.01), ("bf16", 0.01)])
def test_mixed_storage_tip_velocity_report(storage, bound):
    """Mixed storage error against the oracle: tip velocity within 1 %."""
    pb = workload_octant(n=48, steps=400)
    pb.reduce_every = 100
    s = make_gpu(pb, storage)
    s.step(400)
    hist = s.history()
    o = make_oracle(pb)
    tg, to = [], []
    for h in hist:
        o.step(100)
        tg.append(h["tip"][0])
        to.append(o.reduce(pb.centre())[R_TIPX])
    vg, vo = np.diff(tg), np.diff(to)
    rel = np.max(np.abs(vg - vo) / np.abs(vo))
    print("%s tip velocity rel. error %.3e" % (storage, rel))
    assert rel < bound


def _hip_runtime():
    """The HIP runtime the library is linked against (device buffers for the
    device-array calls; a second runtime, such as one bundled with another
    package, would own its allocations and streams separately)."""
    import ctypes
    h = ctypes.CDLL("libamdhip64.so.7")
    h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    h.hipFree.argtypes = [ctypes.c_void_p]
    return h


@pytest.mark.parametrize("storage,dtype", [("f32", "f32"), ("f32", "f64"), ("f16", "f32"), ("f64", "f64")])
def test_device_field_io_matches_host_io(storage, dtype):
    """Fields handed over and read back as device arrays give the same state
    and the same numbers as the host-array calls."""
    import ctypes
    hip = _hip_runtime()
    pb = ragged()
    npdt = np.float32 if dtype == "f32" else np.float64
    host_in = [np.ascontiguousarray(a, dtype=npdt) for a in pb.initial_fields()]
    nbytes = host_in[0].nbytes
    bufs = []
    for _ in range(6):
        p = ctypes.c_void_p()
        assert hip.hipMalloc(ctypes.byref(p), nbytes) == 0
        bufs.append(p)
    try:
        for b, a in zip(bufs[:3], host_in):
            assert hip.hipMemcpy(b, a.ctypes.data_as(ctypes.c_void_p), nbytes, 1) == 0
        host = lbpf.solver_for(pb, storage=storage)
        host.set_fields(*[a.astype(np.float64) for a in host_in])
        devs = lbpf.solver_for(pb, storage=storage)
        devs.set_fields_device(*(b.value for b in bufs[:3]), dtype=dtype)
        host.step(25)
        devs.step(25)
        devs.read_fields_device(*(b.value for b in bufs[3:]), dtype=dtype)
        devs.sync()
        for a, b in zip(fields(host), bufs[3:]):
            out = np.empty(pb.shape, dtype=npdt)
            assert hip.hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), b, nbytes, 2) == 0
            assert np.array_equal(a.astype(npdt), out)
    finally:
        for b in bufs:
            hip.hipFree(b)


def test_separate_lattices_runtime_paths():
    """phi on D3Q19 with U and theta on D3Q7: graph replay, the autotuner
    (which restores the state it found) and checkpoint/restore of the
    population sets of both lattices all give the plain launches' fields bit
    for bit."""
    pb = dataclasses.replace(ragged(), dt=0.11)
    plain = make_gpu(pb, "f32", lattice_ut=7)
    graph = make_gpu(pb, "f32", lattice_ut=7)
    graph.set_graph(4)
    for chunk in (3, 8, 5):
        plain.step(chunk)
        graph.step(chunk)
        for x, y in zip(fields(plain), fields(graph)):
            assert np.array_equal(x, y), chunk
    launches, best = graph.autotune(1)
    assert best > 0 and set(launches) == {"k_phi", "k_ut"}
    for x, y in zip(fields(plain), fields(graph)):
        assert np.array_equal(x, y), "state after autotune"
    pops = [plain.read_populations(f) for f in range(3)]
    assert [p.shape[0] for p in pops] == [19, 7, 7]
    state = fields(plain)
    for s in (plain, graph):
        s.step(12)
    want = fields(plain)
    for x, y in zip(want, fields(graph)):
        assert np.array_equal(x, y), "after autotune, 12 steps"
    r = lbpf.solver_for(pb, storage="f32", lattice_ut=7)
    r.set_fields(*state)
    for f in range(3):
        r.write_populations(f, pops[f])
    r.step(12)
    for x, y in zip(want, fields(r)):
        assert np.array_equal(x, y), "restored"


@pytest.mark.gpu
@pytest.mark.parametrize("storage,over", [("f32", {}), ("f16", {}), ("bf16", {}), ("f64", {}),
                                          ("f32", {"skip_theta": 1}), ("f16", {"skip_U": 1})])
def test_population_writes_leave_other_fields_intact(storage, over):
    """With both transport fields solved, h and f share one device array
    (side by side per direction and node); in the single-field modes each has
    its own.  Writing one field's populations must leave the others' bit for
    bit, and each field must read back exactly what was written, on both
    layouts and every storage type."""
    pb = dataclasses.replace(ragged(), Mcinf=0.0) if over.get("skip_U") else ragged()
    s = lbpf.solver_for(pb, storage=storage, **over)
    s.set_fields(*pb.initial_fields())
    s.step(3)
    rng = np.random.default_rng(11)

    def bits(a):
        return a.view(np.uint8)

    have = [s.read_populations(f) for f in range(3)]
    for f in (1, 2, 0, 1):
        new = rng.integers(0, 256, size=bits(have[f]).shape, dtype=np.uint8).view(have[f].dtype)
        new = new.reshape(have[f].shape)
        s.write_populations(f, new)
        have[f] = new
        for g in range(3):
            assert np.array_equal(bits(s.read_populations(g)), bits(have[g])), (f, g)


@pytest.mark.gpu
def test_autotune_cache(tmp_path):
    """lbpf_autotune_cached: the first call tunes and appends one line, a
    second context of the same configuration takes its launches from that
    line without timing (and steps to the same fields as the tuned one), a
    line that does not parse, names a refused launch or was tuned for other
    kernel sources is skipped, and another domain size is a miss of its
    own."""
    cache = str(tmp_path / "tune.txt")
    pb = ragged()
    a = make_gpu(pb, "f32")
    la, best_a, hit = a.autotune_cached(cache, 1)
    assert not hit and best_a > 0
    lines = open(cache).read().splitlines()
    prefix = "lbpf-autotune-2 k%s " % kernel_build_id()
    assert len(lines) == 1 and lines[0].startswith(prefix) and " q19 qut19 s0 45x23x21 pin0 " in lines[0]
    key = lines[0].split(" pin0 ")[0] + " pin0"
    # a launch the library accepts, but keyed by another kernel build
    other = (32, 16, 8, 0) if tuple(la["k_phi"]) != (32, 16, 8, 0) else (64, 2, 4, 0)
    stale = key.replace(prefix, "lbpf-autotune-2 k0123456789abcdef ") + " %d %d %d %d %d %d %d %d 0.5" % (other + other)
    # a garbled line, a refused launch (a 48x8 tile) and the stale line ahead of the good one
    with open(cache, "w") as fh:
        fh.write(key + " 1 2 3\n")
        fh.write(key + " 48 8 6 1 64 4 6 0 0.5\n")
        fh.write(stale + "\n")
        fh.write(lines[0] + "\n")
    b = make_gpu(pb, "f32")
    lb, best_b, hit = b.autotune_cached(cache, 1)
    assert hit and lb == la and abs(best_b - best_a) <= 1e-6 * best_a
    a.step(10)
    b.step(10)
    for x, y in zip(fields(a), fields(b)):
        assert np.array_equal(x, y)
    c = make_gpu(ragged(n=(37, 21, 19)), "f32")
    _, _, hit = c.autotune_cached(cache, 1)
    assert not hit
    assert len(open(cache).read().splitlines()) == 5


def _mixed_lattice_batch():
    """(problem, lattice_ut) pairs: phi and U/theta lattices mixed within and
    across domains, at dt/tau0 = 0.11 (inside the D3Q7 and D3Q15 windows)."""
    def r(lat, n, seed, **kw):
        return dataclasses.replace(ragged(lat, n, seed=seed, **kw), dt=0.11)
    return [(r(19, (33, 21, 19), 21), 7), (r(15, (40, 17, 24), 22, eps=0.03), 7),
            (r(7, (29, 29, 13), 23), 19), (r(19, (17, 40, 33), 24, aniso=1, eps=0.0, delta=-0.02), 0),
            (r(19, (37, 21, 19), 25, U0=-0.45), 15)]


def test_batch_separate_lattices_match():
    """A batch whose domains put U and theta on another lattice than phi:
    FP64 against the oracle's separate-lattice mode (1e-12), FP32 against
    the domains stepped alone (1e-6, as for one-lattice batches), with graph
    replay."""
    pairs = _mixed_lattice_batch()
    specs = [dict(lbpf.problem_kwargs(p), lattice_ut=lu) for p, lu in pairs]
    b = lbpf.Batch(specs, storage="f64")
    for d, (p, lu) in zip(b.domains, pairs):
        d.set_fields(*p.initial_fields())
    b.step(30)
    for d, (p, lu) in zip(b.domains, pairs):
        o = Oracle(p.nx, p.ny, p.nz, **dict(p.model_kwargs(), lattice_ut=lu))
        o.init(*p.initial_fields())
        o.step(30)
        for x, y in zip(fields(d), o.fields()):
            assert maxabs(x, y) <= 1e-12, (p.lattice, lu)
    b.close()
    b = lbpf.Batch(specs, storage="f32")
    for d, (p, lu) in zip(b.domains, pairs):
        d.set_fields(*p.initial_fields())
    b.set_graph(6)
    b.step(25)
    for d, (p, lu) in zip(b.domains, pairs):
        s = make_gpu(p, "f32", lattice_ut=lu)
        s.step(25)
        for x, y in zip(fields(s), fields(d)):
            assert maxabs(x, y) <= 1e-6, (p.lattice, lu)
        s.close()
    b.close()
