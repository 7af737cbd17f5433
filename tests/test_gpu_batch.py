"""Batched PCG (lockstep members under a hipGraph, per-member device stopping test) and the
launch-shape autotuner, checked against single solves and the oracle.

Bounds: a member of the batch performs the same kernels on the same data as the
single solve, so iteration counts are equal and iterates agree up to the order of
floating-point atomic additions in the operator (x relative difference below 1e-10).
With the FP32 cycle those additions happen in FP32 inside the preconditioner, so two
runs of the same solve differ at the 1e-7 level per application: iteration counts may
then differ by one at the stopping threshold, both solutions meet the 1e-8 residual
bound, and x agrees to 1e-6.  Launch shapes change no arithmetic either.
"""
import numpy as np
import pytest

from paper_2107_14758_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def vsr():
    from paper_2107_14758_amd import vsr as v
    v.lib()
    return v


# (n per axis, p, jitter, lognormal kappa): sizes, degrees and geometry all differ
MEMBERS = [((2, 2, 2), 3, 0.0, False), ((3, 3, 3), 4, 0.15, True), ((2, 3, 2), 5, 0.0, True),
           ((4, 4, 4), 2, 0.2, False), ((3, 3, 3), 6, 0.0, False), ((2, 2, 2), 7, 0.15, True),
           ((3, 2, 4), 4, 0.0, False)]


def member_problem(shape, p, jitter, logn, seed):
    rng = np.random.default_rng(seed)
    V = inputs.cube_vertices(*shape)
    if jitter:
        V = inputs.jitter_vertices(V, jitter, rng)
    kappa = inputs.lognormal_kappa(*shape, rng) if logn else None
    q = inputs.quadrature_points_per_dir(p)
    f = inputs.rhs_samples(int(np.prod(shape)), q ** 3, rng)
    return dict(vertices=V, p=p, kappa=kappa), f


def rhs(prob, f):
    b = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
    prob.load_vector(torch.tensor(f, dtype=torch.float64, device="cuda"), b)
    return b


def rel(a, b):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


@pytest.mark.parametrize("eager,relax_fp32", [(False, False), (False, True), (True, False)])
def test_batch_matches_single_solves(vsr, eager, relax_fp32):
    say(f"case batch eager={eager} fp32={relax_fp32}")
    probs, fs = zip(*[member_problem(*m, seed=10 + i) for i, m in enumerate(MEMBERS)])
    B = vsr.Batch(list(probs), relax_fp32=relax_fp32, seed=0, batch_eager=eager, batch_streams=3)
    bs = [rhs(m, f) for m, f in zip(B.members, fs)]
    for rep in range(2):   # the second solve replays the recorded iteration with new right-hand sides
        if rep:
            bs = [b * (1.0 + 0.5 * i) for i, b in enumerate(bs)]
        xs = [torch.zeros_like(b) for b in bs]
        infos = B.pcg_solve(bs, xs)
        for i, (m, b, x, info) in enumerate(zip(B.members, bs, xs, infos)):
            x1 = torch.zeros_like(b)
            ref = m.pcg_solve(b, x1)
            say(f"  rep {rep} member {i}: n={m.n} its {info['iterations']} vs {ref['iterations']}, "
                f"true res {info['true_rel_residual']:.2e}")
            assert info["converged"] == 1 and info["true_rel_residual"] <= 1.0001e-8
            say(f"    x rel diff {rel(x, x1):.1e}, residual ratio {info['rel_residual'] / ref['rel_residual']:.8f}")
            if relax_fp32:
                assert abs(info["iterations"] - ref["iterations"]) <= 1 and rel(x, x1) < 1e-6
            else:
                assert info["iterations"] == ref["iterations"]
                assert abs(info["rel_residual"] / ref["rel_residual"] - 1) < 1e-6
                assert rel(x, x1) < 1e-10
    B.close()


def test_batch_member_matches_oracle(vsr):
    say("case batch oracle")
    from oracle.operator import Discretization
    from oracle.fdm1d import setup_1d
    from oracle.solver import Solver
    probs, fs = zip(*[member_problem(*m, seed=20 + i) for i, m in enumerate(MEMBERS[:3])])
    B = vsr.Batch(list(probs), seed=0)
    bs = [rhs(m, f) for m, f in zip(B.members, fs)]
    xs = [torch.zeros_like(b) for b in bs]
    infos = B.pcg_solve(bs, xs)
    for i in (0, 2):
        d = probs[i]
        disc = Discretization(d["vertices"], d["p"], d["kappa"])
        od = setup_1d(d["p"])
        b = bs[i].cpu().numpy()
        x, its = Solver(disc, od, seed=0).pcg(b, rtol=1e-8)
        say(f"  member {i}: its {infos[i]['iterations']} oracle {its}")
        assert infos[i]["iterations"] == its
        assert np.linalg.norm(xs[i].cpu().numpy() - x) / np.linalg.norm(x) < 1e-9
    B.close()


def test_batch_zero_rhs_and_iteration_cap(vsr):
    say("case batch stopping")
    probs, fs = zip(*[member_problem(*m, seed=30 + i) for i, m in enumerate(MEMBERS[:3])])
    B = vsr.Batch(list(probs), seed=0, max_iterations=3)
    bs = [rhs(m, f) for m, f in zip(B.members, fs)]
    bs[1].zero_()
    xs = [torch.full_like(b, 7.0) for b in bs]
    infos = B.pcg_solve(bs, xs, raise_on_noconv=False)
    assert infos[0]["status"] == vsr.VSR_ENOCONV
    assert infos[1]["converged"] == 1 and infos[1]["iterations"] == 0 and float(xs[1].abs().max()) == 0.0
    for i in (0, 2):
        assert infos[i]["converged"] == 0 and infos[i]["iterations"] == 3
        x1 = torch.zeros_like(bs[i])
        ref = B.members[i].pcg_solve(bs[i], x1, raise_on_noconv=False)
        assert ref["iterations"] == 3 and rel(xs[i], x1) < 1e-10
    B.close()


@pytest.mark.parametrize("p,jitter,relax_fp32", [(4, 0.0, True), (7, 0.0, False), (5, 0.2, True), (3, 0.0, False),
                                                 (6, 0.15, False)])
def test_every_launch_shape_gives_the_same_solve(vsr, p, jitter, relax_fp32):
    say(f"case shapes p={p} jitter={jitter} fp32={relax_fp32}")
    d, f = member_problem((3, 3, 3), p, jitter, False, seed=40 + p)
    prob = vsr.Problem(d["vertices"], p, relax_fp32=relax_fp32, seed=0)
    b = rhs(prob, f)
    x0 = torch.zeros_like(b)
    ref = prob.pcg_solve(b, x0)
    assert prob.tuning() == (1, 4, 4, 0, 0, 256)
    for shapes in [(2, 2, 4, 1, 2, 512), (4, 4, 16, 2, 1, 256), (4, 2, 8, 2, 2, 1024), (1, 4, 16, 1, 1, 512),
                   (1, 1, 4, 0, 0, 1024)]:
        prob.set_tuning(shapes)
        x = torch.zeros_like(b)
        info = prob.pcg_solve(b, x)
        say(f"  shapes {shapes}: its {info['iterations']} (default {ref['iterations']}) rel {rel(x, x0):.1e}")
        if relax_fp32:
            assert abs(info["iterations"] - ref["iterations"]) <= 1 and rel(x, x0) < 1e-6
        else:
            assert info["iterations"] == ref["iterations"] and rel(x, x0) < 1e-10
    with pytest.raises(vsr.VsrError):
        prob.set_tuning((3, 1, 8, 0, 0, 256))
    with pytest.raises(vsr.VsrError):
        prob.set_tuning((1, 1, 8, 0, 0, 300))
    with pytest.raises(vsr.VsrError):
        prob.set_tuning((1, 1, 16, 0, 0, 1024))
    prob.close()


def test_autotune_and_cache_file(vsr, tmp_path):
    say("case autotune")
    cache = tmp_path / "tune.txt"
    d, f = member_problem((4, 4, 4), 4, 0.0, False, seed=50)
    prob = vsr.Problem(d["vertices"], 4, relax_fp32=True, seed=0, autotune=True, tune_cache=str(cache))
    t = prob.tuning()
    say(f"  tuned shapes {t}")
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and " p=4 prec=f32 op=kron " in lines[0]
    assert lines[0].endswith(f"cpw64={t[0]} cpw32={t[1]} patch_unroll={t[2]} split64={t[3]} split32={t[4]} "
                             f"patch_threads={t[5]}")
    b = rhs(prob, f)
    x = torch.zeros_like(b)
    info = prob.pcg_solve(b, x)
    plain = vsr.Problem(d["vertices"], 4, relax_fp32=True, seed=0)
    x1 = torch.zeros_like(b)
    ref = plain.pcg_solve(b, x1)
    assert abs(info["iterations"] - ref["iterations"]) <= 1 and rel(x, x1) < 1e-6
    # a second problem with the same key takes the cached shapes and appends nothing
    again = vsr.Problem(d["vertices"], 4, relax_fp32=True, seed=0, autotune=True, tune_cache=str(cache))
    assert again.tuning() == t and len(cache.read_text().splitlines()) == 1
    for q in (prob, plain, again):
        q.close()


@pytest.mark.parametrize("relax_fp32", [False, True])
def test_single_solve_graph_and_host_driven_agree(vsr, relax_fp32):
    """vsr_pcg_solve replays a recorded iteration with the stop taken on the device unless
    profiling is on, when the host drives every iteration; both give the same solve."""
    say(f"case single-solve paths fp32={relax_fp32}")
    d, f = member_problem((3, 3, 3), 5, 0.15, True, seed=60)
    prob = vsr.Problem(d["vertices"], 5, kappa=d["kappa"], relax_fp32=relax_fp32, seed=0)
    b = rhs(prob, f)
    x_graph, x_host = torch.zeros_like(b), torch.zeros_like(b)
    info_g = prob.pcg_solve(b, x_graph)
    prob.set_profiling(True)
    info_h = prob.pcg_solve(b, x_host)
    prob.set_profiling(False)
    launches, total_ms, _ = prob.kernel_stats()
    say(f"  graph {info_g['iterations']} its, host {info_h['iterations']} its, rel {rel(x_graph, x_host):.1e}, "
        f"{launches} profiled patch launches")
    assert launches == info_h["iterations"] * 2 and total_ms > 0   # two relaxations per cycle
    tol = 1e-6 if relax_fp32 else 1e-10
    assert abs(info_g["iterations"] - info_h["iterations"]) <= (1 if relax_fp32 else 0)
    assert rel(x_graph, x_host) < tol
    x_again = torch.zeros_like(b)
    info_again = prob.pcg_solve(b * 2.0, x_again)   # the recorded iteration is reused
    assert info_again["iterations"] == info_g["iterations"] or relax_fp32
    assert rel(x_again, 2.0 * x_graph) < tol
    prob.close()


@pytest.mark.parametrize("relax_fp32", [False, True])
def test_shared_factors_give_the_same_solve(vsr, relax_fp32):
    """With share_factors every interior star of a uniform Cartesian mesh with constant kappa
    uses one stored factor (and the boundary classes one each); the solve is unchanged."""
    say(f"case shared factors fp32={relax_fp32}")
    d, f = member_problem((4, 4, 4), 5, 0.0, False, seed=70)
    own = vsr.Problem(d["vertices"], 5, relax_fp32=relax_fp32, seed=0)
    shared = vsr.Problem(d["vertices"], 5, relax_fp32=relax_fp32, seed=0, share_factors=True)
    npatch, entries_own = own.factor_info()
    npatch2, entries_shared = shared.factor_info()
    say(f"  {npatch} patches, stored factor entries {entries_own} -> {entries_shared}")
    assert npatch == npatch2 and entries_shared < entries_own / 10
    # the shared factor equals each star's own up to rounding of the cell scalings
    assert abs(own.damping()[0] / shared.damping()[0] - 1) < (1e-5 if relax_fp32 else 1e-9)
    b = rhs(own, f)
    x1, x2 = torch.zeros_like(b), torch.zeros_like(b)
    i1, i2 = own.pcg_solve(b, x1), shared.pcg_solve(b, x2)
    tol = 1e-6 if relax_fp32 else 1e-10
    assert abs(i1["iterations"] - i2["iterations"]) <= (1 if relax_fp32 else 0)
    assert rel(x2, x1) < tol
    # a jittered mesh has no two identical stars
    dj, _ = member_problem((3, 3, 3), 4, 0.15, True, seed=71)
    pj = vsr.Problem(dj["vertices"], 4, kappa=dj["kappa"], seed=0, share_factors=True)
    pj_own = vsr.Problem(dj["vertices"], 4, kappa=dj["kappa"], seed=0)
    assert pj.factor_info() == pj_own.factor_info()
    for q in (own, shared, pj, pj_own):
        q.close()


def test_retuning_a_member_between_batch_solves(vsr):
    """A member retuned after the batch recorded its iteration: the next batch solve records the
    iteration again with the new launch shapes and still matches the member's single solve."""
    say("case batch retune")
    probs, fs = zip(*[member_problem(*m, seed=40 + i) for i, m in enumerate(MEMBERS[:3])])
    B = vsr.Batch(list(probs), relax_fp32=False, seed=0, batch_streams=2)
    bs = [rhs(m, f) for m, f in zip(B.members, fs)]
    xs = [torch.zeros_like(b) for b in bs]
    B.pcg_solve(bs, xs)
    m = B.members[1]
    old = m.tuning()
    new = (2, 2, 8 if old[2] != 8 else 4, 1 if old[3] != 1 else 2, 2 if old[4] != 2 else 1, 512 if old[5] != 512 else 256)
    m.set_tuning(new)
    assert m.tuning() == new
    xs = [torch.zeros_like(b) for b in bs]
    infos = B.pcg_solve(bs, xs)
    for i, (mm, b, x, info) in enumerate(zip(B.members, bs, xs, infos)):
        x1 = torch.zeros_like(b)
        ref = mm.pcg_solve(b, x1)
        say(f"  member {i}: its {info['iterations']} vs {ref['iterations']}, x rel diff {rel(x, x1):.1e}")
        assert info["converged"] == 1 and info["iterations"] == ref["iterations"]
        assert rel(x, x1) < 1e-10
    B.close()
