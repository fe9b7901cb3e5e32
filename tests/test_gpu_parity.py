"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same seeded
inputs. Leaf sets bit-exact (near-threshold flips reported), moments within 1e-12 relative
on FP64, FP32 storage within 1e-5 relative plus the eps bound, eps = 0 equal to the uniform
scheme to 1e-13. Sizes run from a few cells per level (partial 64-bit words) to the full
workload sizes (J = 14 and 16)."""

import sys

import numpy as np
import pytest

import workloads as W
from oracle import metrics
from oracle.lattice import scheme_from_params
from oracle.reference import UniformLBM
from paper_2102_12163_amd import mrlbm

from gpu_helpers import compare_run, first_divergence, make_oracle, rel_err

pytestmark = pytest.mark.gpu


def announce(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def run_pair(p, mc, nsteps, every, label):
    """The GPU run and the oracle side by side, compared every ``every`` steps; a leaf-set
    difference fails, with the step where the trees first diverged located by a re-run."""
    announce(label, "J", p["jmax"], "steps", nsteps)
    run = mrlbm.MRLBM(p, mc)
    ora = make_oracle(p, mc)
    done = 0
    try:
        while done < nsteps:
            k = min(every, nsteps - done)
            run.step(k)
            ora.step(k)
            done += k
            upto = done
            compare_run(run, ora, f"{label} step {done}",
                        locate=lambda: first_divergence(lambda: mrlbm.MRLBM(p, mc), p, mc, upto))
        st = run.stats()
        assert st["steps"] == done
        assert st["leaf_updates"] == ora.leaf_updates
    finally:
        run.close()


KINDS = ["advection", "burgers", "burgers_d1q2", "shallow", "shallow_d1q3", "shallow_d1q5", "euler"]


@pytest.mark.parametrize("kind", KINDS)
def test_step_parity_small(kind):
    for seed in (0, 1):
        p, mc = W.small_case(kind, seed=seed, jmax=9)
        run_pair(p, mc, 60, 10, f"{kind} seed {seed}")


@pytest.mark.parametrize("kind", KINDS)
def test_step_parity_tiny_levels(kind):
    """J = 5: every level fits in one partial 64-bit word."""
    p, mc = W.small_case(kind, seed=3, jmax=5, eps=1e-3)
    run_pair(p, mc, 30, 3, f"{kind} tiny")


@pytest.mark.parametrize("gamma", [2, 3])
@pytest.mark.parametrize("bc", [0, 1])
def test_step_parity_wider_prediction(gamma, bc):
    p, mc = W.advection(4, jmax=9, eps=1e-4)
    p["gamma"], p["jmin"], p["bc"] = gamma, 3, bc
    run_pair(p, mc, 40, 10, f"gamma {gamma} bc {bc}")


def test_step_parity_mu_bar_and_clamp():
    p, mc = W.burgers(2, jmax=9, eps=1e-4)
    p["mu_bar"], p["bc"] = 2, 1
    run_pair(p, mc, 40, 10, "mu_bar 2 clamp")


@pytest.mark.parametrize("kind", KINDS)
def test_step_parity_coarsest_level_zero(kind):
    """J_min = 0: the coarsest level is one cell (under clamp; a periodic coarsest level needs
    2 gamma + 1 cells). Every family against the oracle, and gamma = 2 on the first."""
    p, mc = W.small_case(kind, seed=3, jmax=9)
    p["jmin"], p["bc"] = 0, 1  # clamp
    run_pair(p, mc, 60, 10, f"{kind} jmin 0")
    if kind == KINDS[0]:
        p["gamma"] = 2
        run_pair(p, mc, 40, 10, f"{kind} jmin 0 gamma 2")


@pytest.mark.parametrize("kind", KINDS)
def test_eps_zero_is_uniform_scheme(kind):
    p, mc = W.small_case(kind, seed=1, jmax=8)
    p["eps"] = 0.0
    announce("eps0", kind)
    run = mrlbm.MRLBM(p, mc)
    run.step(40)
    ref = UniformLBM(scheme_from_params(p), p["jmax"], p["bc"], mc).step(40)
    got = run.moments(mrlbm.FINEST)
    want = ref.conserved()
    assert run.stats()["leaves"] == 2 ** p["jmax"]
    assert rel_err(got, want) <= 1e-13
    run.close()


@pytest.mark.parametrize("kind", ["advection", "burgers", "euler"])
def test_adapt_only_parity(kind):
    p, mc = W.small_case(kind, seed=2, jmax=10, eps=1e-3)
    announce("adapt", kind)
    run = mrlbm.MRLBM(p, mc)
    ora = make_oracle(p, mc)
    for _ in range(2):
        run.adapt()
        ora.adapt()
        # the handle's statistics follow an adaptation (before any query refreshes them)
        assert run.stats()["leaves"] == ora.n_leaves()
        lv, ix = run.leaves()
        olv, oix = ora.leaf_list()
        assert np.array_equal(lv, olv) and np.array_equal(ix, oix)
        pops = run.populations()
        assert rel_err(pops, ora.leaf_populations()) <= 1e-14
    run.close()


@pytest.mark.parametrize("kind", ["advection", "shallow", "euler"])
def test_finest_reconstruction_parity(kind):
    p, mc = W.small_case(kind, seed=5, jmax=10, eps=1e-4)
    announce("finest", kind)
    run = mrlbm.MRLBM(p, mc)
    ora = make_oracle(p, mc)
    run.step(25)
    ora.step(25)
    assert rel_err(run.moments(mrlbm.FINEST), ora.finest_conserved()) <= 1e-12
    run.close()


def test_edge_cases():
    # J_min == J: nothing to adapt, the uniform scheme on 2^J cells
    p, mc = W.advection(0, jmax=6)
    p["jmin"] = 6
    announce("edge jmin==jmax")
    run_pair(p, mc, 20, 5, "jmin==jmax")
    # eps so large that everything coarsens to J_min
    p, mc = W.burgers(1, jmax=8)
    p["eps"] = 1e3
    run_pair(p, mc, 10, 5, "huge eps")
    run = mrlbm.MRLBM(p, mc)
    run.step(3)
    assert run.stats()["leaves"] == 2 ** p["jmin"]
    run.close()
    # zero steps is a no-op, negative steps are rejected
    run = mrlbm.MRLBM(p, mc)
    run.step(0)
    assert run.stats()["steps"] == 0
    assert mrlbm.lib().mrlbm_step(run.h, -1) == mrlbm.EINVAL
    assert mrlbm.lib().mrlbm_moments(run.h, 7, None, 0, None) == mrlbm.EINVAL
    import ctypes
    n = ctypes.c_int64()
    buf = np.empty(1)
    rc = mrlbm.lib().mrlbm_moments(run.h, mrlbm.FINEST, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1,
                                   ctypes.byref(n))
    assert rc == mrlbm.ECAPACITY and n.value == 2 ** p["jmax"]
    run.close()


@pytest.mark.parametrize("kind", ["burgers", "shallow", "euler"])
def test_fp32_storage_within_bound(kind):
    """FP32 state, FP64 details: within 1e-5 relative plus the eps bound of the FP64 run."""
    p, mc = W.small_case(kind, seed=0, jmax=10, eps=1e-4)
    p32 = dict(p, precision=mrlbm.FP32_STORAGE)
    announce("fp32", kind)
    n = 100
    run = mrlbm.MRLBM(p32, mc)
    run.step(n)
    ora = make_oracle(p, mc).step(n)
    ref = UniformLBM(scheme_from_params(p), p["jmax"], p["bc"], mc).step(n)
    m32 = run.moments(mrlbm.FINEST)
    m64 = ora.finest_conserved()
    d64 = metrics.delta(ref.conserved(), m64, p["x_min"], p["x_max"])
    d3264 = metrics.delta(m64, m32, p["x_min"], p["x_max"])
    norm = metrics.delta(np.zeros_like(m64), m64, p["x_min"], p["x_max"])
    for c in range(m64.shape[0]):
        assert d3264[c] <= 1e-5 * norm[c] + 2.0 * max(d64[c], p["eps"]), (c, d3264, d64)
    run.close()


def test_batch_equals_single_runs():
    """Runs of a batch (uneven J, eps, physics) give bit-identical results to the same runs
    created alone, and match the oracle."""
    cases = [W.batch_instance(s, steps=0) for s in range(6)]
    ps = [c[0] for c in cases]
    ms = [c[1] for c in cases]
    announce("batch", [p["jmax"] for p in ps])
    b = mrlbm.Batch(ps, ms)
    b.step(30)
    b.step(30)
    for i, (p, mc) in enumerate(cases):
        single = mrlbm.MRLBM(p, mc)
        single.step(60)
        assert np.array_equal(b.moments(i), single.moments())
        lv, ix = b.leaves(i)
        slv, six = single.leaves()
        assert np.array_equal(lv, slv) and np.array_equal(ix, six)
        single.close()
        ora = make_oracle(p, mc).step(60)
        olv, oix = ora.leaf_list()
        assert np.array_equal(lv, olv) and np.array_equal(ix, oix)
        assert rel_err(b.moments(i), ora.leaf_conserved()) <= 1e-12
    assert b.total_updates() == sum(b.stats(i)["leaf_updates"] for i in range(len(cases)))
    b.close()


def test_batch_of_uneven_coarsest_levels():
    """Runs whose J_min differ (0 to 3, clamp) share one launch, each with its own LDS layout:
    the batch equals the oracle run by run, on chip and on the HBM path (capacity 0)."""
    cases = []
    for s_, jmin in enumerate((0, 1, 2, 3, 0, 2)):
        p, mc = W.batch_instance(s_, steps=0)
        p["jmin"], p["bc"] = jmin, 1  # clamp
        cases.append((p, mc))
    ps, ms = [c[0] for c in cases], [c[1] for c in cases]
    announce("batch jmin", [(p["jmin"], p["jmax"]) for p in ps])
    for cap in (-1, 0):
        b = mrlbm.Batch(ps, ms)
        if cap == 0:
            b.set_capacity(0)
        b.step(40)
        for i, (p, mc) in enumerate(cases):
            ora = make_oracle(p, mc).step(40)
            lv, ix = b.leaves(i)
            olv, oix = ora.leaf_list()
            assert np.array_equal(lv, olv) and np.array_equal(ix, oix), (cap, i)
            assert rel_err(b.moments(i), ora.leaf_conserved()) <= 1e-12, (cap, i)
        b.close()


def test_full_size_burgers_d1q3():
    """The D1Q3 Burgers workload at its full size (J = 14, 16384 finest cells)."""
    p, mc = W.burgers(0, jmax=14, eps=1e-4, s=1.9)
    run_pair(p, mc, 120, 40, "burgers J14")


def test_full_size_advection_2000_steps():
    p, mc = W.advection(0, jmax=10)
    run_pair(p, mc, 2000, 500, "advection J10")


def test_full_size_shallow_water_j16():
    p, mc = W.shallow(0, jmax=16)
    run_pair(p, mc, 30, 15, "shallow J16")


def test_full_size_shallow_water_d1q5_j16():
    """D1Q5 (Sec. 5.2: velocities 0, +-lambda, +-2 lambda, alpha = beta = 1, s3 = s4 = 1) on
    the dam break at J = 16: the two-cell stream (sigma = 2) and rule (a) with sigma = 2,
    bit-exact with the oracle over 300 steps."""
    p, mc = W.shallow(0, jmax=16, scheme=W.D1Q5, s=1.5)
    run_pair(p, mc, 300, 100, "shallow d1q5 J16")


@pytest.mark.parametrize("bc", [0, 1])
def test_d1q5_wider_prediction_and_both_boundaries(bc):
    """D1Q5 with gamma = 2 (a nine-cell reconstruction window) on both boundary readings, the
    two-cell stream's clamped cells at the domain ends included."""
    p, mc = W.small_case("shallow_d1q5", seed=6, jmax=9, eps=1e-4)
    p = dict(p, gamma=2, jmin=3, bc=bc)
    run_pair(p, mc, 40, 10, f"d1q5 gamma 2 bc {bc}")


def test_full_size_euler_j14():
    p, mc = W.euler(0, jmax=14)
    run_pair(p, mc, 60, 30, "euler J14")


@pytest.mark.parametrize("cap", [0, 120, 400])
def test_onchip_capacity_does_not_change_results(cap):
    """Runs whose trees live in HBM (capacity 0) or switch between LDS and HBM from step to
    step (small capacities) give the same bits as the on-chip runs and the oracle."""
    cases = [W.small_case(k, seed=7, jmax=10, eps=1e-4) for k in ("advection", "burgers_d1q2")]
    announce("capacity", cap)
    for p, mc in cases:
        b = mrlbm.Batch([p], [mc])
        b.set_capacity(cap)
        assert b.get_capacity() == cap
        ref = mrlbm.Batch([p], [mc])
        ora = make_oracle(p, mc)
        for _ in range(4):
            b.step(15)
            ref.step(15)
            ora.step(15)
            assert np.array_equal(b.moments(0), ref.moments(0))
            lv, ix = b.leaves(0)
            olv, oix = ora.leaf_list()
            assert np.array_equal(lv, olv) and np.array_equal(ix, oix)
            assert rel_err(b.moments(0), ora.leaf_conserved()) <= 1e-12
        b.close()
        ref.close()


def test_tuner_keeps_state_and_results():
    """The launch-shape tuner restores every run after its trials: a tuned batch continues
    bit for bit like an untuned one."""
    cases = [W.batch_instance(s, steps=0) for s in range(10)]
    announce("tuner")
    a = mrlbm.Batch([c[0] for c in cases], [c[1] for c in cases])
    b = mrlbm.Batch([c[0] for c in cases], [c[1] for c in cases])
    a.step(10)
    b.step(10)
    threads, cells = a.tune(5)
    if a.get_classes():  # the tuner chose launch classes
        assert (threads, cells) == (0, 0)
    else:
        assert threads in (128, 256, 384, 512) and cells >= 0
    assert all(a.stats(i)["steps"] == 10 for i in range(len(cases)))
    a.step(25)
    b.step(25)
    for i in range(len(cases)):
        assert np.array_equal(a.moments(i), b.moments(i))
    a.close()
    b.close()


def test_block_size_does_not_change_results():
    """FP32-storage runs give the same bits at 128 and 384 threads per workgroup as at 512
    (every thread count reaches the same per-cell arithmetic)."""
    cases = [W.batch_instance(s, steps=0) for s in range(8)]
    ps = [dict(c[0], precision=mrlbm.FP32_STORAGE) for c in cases]
    ms = [c[1] for c in cases]
    announce("block sizes", [p["jmax"] for p in ps])
    ref = mrlbm.Batch(ps, ms)
    ref.set_block(512)
    ref.step(40)
    for nt in (384, 128):
        b = mrlbm.Batch(ps, ms)
        b.set_block(nt)
        assert b.get_block() == nt
        b.step(25)
        b.step(15)
        for i in range(len(ps)):
            assert np.array_equal(b.moments(i), ref.moments(i)), (nt, i)
            lv, ix = b.leaves(i)
            rlv, rix = ref.leaves(i)
            assert np.array_equal(lv, rlv) and np.array_equal(ix, rix), (nt, i)
        b.close()
    ref.close()


def test_schedule_does_not_change_results():
    """The workgroup-to-run schedule only moves runs between workgroups."""
    cases = [W.batch_instance(s, steps=0) for s in range(24)]
    announce("schedule", len(cases))
    ps, ms = [c[0] for c in cases], [c[1] for c in cases]
    a = mrlbm.Batch(ps, ms)
    b = mrlbm.Batch(ps, ms)
    try:
        a.step(10)
        b.step(10)
        assert b.get_schedule() == 0
        b.set_schedule(5)
        assert b.get_schedule() == 5
        a.step(25)
        b.step(25)
        b.set_schedule(len(cases))  # heaviest first
        assert b.get_schedule() == len(cases)
        a.step(4)
        b.step(4)
        b.set_schedule(1)
        b.set_launch_steps(3)  # 7 steps as launches of 3, 3, 1
        a.step(7)
        b.step(7)
        for i in range(len(cases)):
            la, ia = a.leaves(i)
            lb, ib = b.leaves(i)
            assert np.array_equal(la, lb) and np.array_equal(ia, ib), i
            assert np.array_equal(a.moments(i), b.moments(i)), i
            assert a.stats(i)["leaf_updates"] == b.stats(i)["leaf_updates"], i
    finally:
        a.close()
        b.close()


def test_bench_workload_in_bench_launch_configuration():
    """The full Burgers batch of the benchmark (510 runs, J = 14) in the launch configuration
    the benchmark times (512 threads, on-chip capacity 1148 cells, heavy/light schedule
    set after a warmup, runs restored to t = 0, the timed steps as one launch): sampled runs
    against the oracle, the rest against a batch with the default launch shape (bit for
    bit)."""
    cases = []
    for s in (1.5, 1.9):
        for eps in (1e-2, 1e-3, 1e-4):
            for seed in range(85):
                cases.append(W.burgers(seed, jmax=14, eps=eps, s=s))
    announce("bench batch", len(cases))
    ps, ms = [c[0] for c in cases], [c[1] for c in cases]
    b = mrlbm.Batch(ps, ms)
    ref = mrlbm.Batch(ps, ms)
    try:
        b.set_block(512)
        b.set_capacity(1148)
        b.checkpoint()
        b.step(113)
        b.set_schedule(256)
        b.restore()
        nsteps = 226
        b.step(nsteps)
        ref.step(nsteps)
        for i in (0, 170, 254, 425, 509):  # light and heavy runs of both relaxation rates
            ora = make_oracle(ps[i], ms[i]).step(nsteps)
            lv, ix = b.leaves(i)
            olv, oix = ora.leaf_list()
            assert np.array_equal(lv, olv) and np.array_equal(ix, oix), i
            assert rel_err(b.moments(i), ora.leaf_conserved()) <= 1e-12, i
        for i in range(0, len(cases), 17):
            assert np.array_equal(b.moments(i), ref.moments(i)), i
        assert b.total_updates() == ref.total_updates()
    finally:
        b.close()
        ref.close()


def test_launch_classes_do_not_change_results():
    """Runs split into launch classes by j_max (each class its own grid, workgroup size and
    on-chip capacity, the class grids side by side) give the bits of the single launch: graph
    and direct launches, chunked launches, the oracle on one run per class; the tuner picks
    a single launch or classes and keeps the results; bad class sets are refused."""
    cases = [W.batch_instance(s, steps=0) for s in range(40)]
    ps, ms = [c[0] for c in cases], [c[1] for c in cases]
    announce("launch classes", sorted(p["jmax"] for p in ps))
    a = mrlbm.Batch(ps, ms)
    b = mrlbm.Batch(ps, ms)
    try:
        b.set_classes([10, 12, 14], [256, 512, 512], [8, 4, 2])
        cl = b.get_classes()
        assert len(cl) == 3 and sum(c[0] for c in cl) == len(cases)
        assert sum(c[0] for c in cl[:1]) == sum(p["jmax"] <= 10 for p in ps)
        a.step(30)
        b.step(30)                       # graph launch
        b.set_launch_steps(7)            # 20 steps as launches of 7, 7, 6
        a.step(20)
        b.step(20)
        for i in range(len(cases)):
            la, ia = a.leaves(i)
            lb, ib = b.leaves(i)
            assert np.array_equal(la, lb) and np.array_equal(ia, ib), i
            assert np.array_equal(a.moments(i), b.moments(i)), i
        assert a.total_updates() == b.total_updates()
        b.set_launch_steps(0)
        ms_ = b.step_timed(5)
        a.step(5)
        assert ms_ > 0 and a.total_updates() == b.total_updates()
        for j_lo, j_hi in ((8, 10), (11, 12), (13, 14)):
            i = next(k for k, p in enumerate(ps) if j_lo <= p["jmax"] <= j_hi)
            ora = make_oracle(ps[i], ms[i]).step(55)
            lv, ix = b.leaves(i)
            olv, oix = ora.leaf_list()
            assert np.array_equal(lv, olv) and np.array_equal(ix, oix), i
            assert rel_err(b.moments(i), ora.leaf_conserved()) <= 1e-12, i
        for bad in (([14, 12], [512, 512], [2, 4]), ([12], [512], [2]), ([14], [100], [2]), ([14], [512], [0])):
            with pytest.raises(mrlbm.MRLBMError):
                b.set_classes(*bad)
        with pytest.raises(mrlbm.MRLBMError):
            b.set_block(256)  # each class has its own shape
        with pytest.raises(mrlbm.MRLBMError):
            b.set_capacity(100)
        u_before = b.total_updates()
        tb, tc = b.tune(3)
        assert (tb, tc) == (0, 0) if b.get_classes() else tb in (128, 256, 384, 512)
        assert b.total_updates() == u_before  # the trials were undone
        b.set_classes()
        b.set_classes([14], [512], [2])
        with pytest.raises(mrlbm.MRLBMError):
            b.set_predictor(None, mrlbm.PRED_RECORD, sample_capacity=10)
        b.set_classes()
        assert b.get_classes() == []
    finally:
        a.close()
        b.close()


def test_checkpoint_restore_repeats_the_same_steps():
    """Steps taken after a restore give what the same steps gave after the checkpoint (bit
    for bit, statistics included); restore without a checkpoint is an error."""
    cases = [W.batch_instance(s, steps=0) for s in range(12)]
    announce("checkpoint", len(cases))
    ps, ms = [c[0] for c in cases], [c[1] for c in cases]
    b = mrlbm.Batch(ps, ms)
    try:
        with pytest.raises(mrlbm.MRLBMError):
            b.restore()
        b.step(9)
        b.checkpoint()
        at = [b.stats(i) for i in range(len(cases))]
        b.step(31)
        first = [(b.leaves(i), b.moments(i), b.stats(i)) for i in range(len(cases))]
        b.restore()
        assert [b.stats(i) for i in range(len(cases))] == at
        b.set_launch_steps(8)  # the repeat as launches of 8, 8, 8, 7 steps
        b.step(31)
        for i, ((lv, ix), m, st) in enumerate(first):
            lv2, ix2 = b.leaves(i)
            assert np.array_equal(lv, lv2) and np.array_equal(ix, ix2), i
            assert np.array_equal(m, b.moments(i)), i
            assert b.stats(i) == st, i
        b.restore()  # the checkpoint stays until the next one
        assert [b.stats(i) for i in range(len(cases))] == at
    finally:
        b.close()


def test_batched_ensemble_at_full_size():
    """The batched ensemble at its full size (4096 instances, J uniform in 8..14, advection
    and Burgers, eps in {1e-3, 1e-4}) in the tuner's launch shape, its 512 steps as one
    launch: one sampled instance per J_max against the oracle (leaves bit for bit, moments
    to 1e-12)."""
    cases = [W.batch_instance(s, steps=0) for s in range(4096)]
    announce("ensemble", len(cases))
    ps, ms = [c[0] for c in cases], [c[1] for c in cases]
    b = mrlbm.Batch(ps, ms)
    try:
        b.tune(8)
        nsteps = 512
        b.step(nsteps)
        picked = {}
        for i, p in enumerate(ps):
            picked.setdefault(p["jmax"], i)
        assert sorted(picked) == list(range(8, 15))
        for j, i in sorted(picked.items()):
            announce("ensemble instance", i, "J", j)
            ora = make_oracle(ps[i], ms[i]).step(nsteps)
            lv, ix = b.leaves(i)
            olv, oix = ora.leaf_list()
            assert np.array_equal(lv, olv) and np.array_equal(ix, oix), i
            assert rel_err(b.moments(i), ora.leaf_conserved()) <= 1e-12, i
        assert all(b.stats(i)["steps"] == nsteps for i in range(0, len(cases), 97))
    finally:
        b.close()


def test_bench_workload_whole_run_sampled():
    """The benchmark's timed region in full: the 510-run Burgers batch from t = 0 to T = 0.4
    (3277 steps) as one launch at on-chip capacity 999, where the heaviest trees outgrow the
    LDS at times and those steps take the HBM path; the heaviest run of each eps against the
    oracle at the end (leaves bit for bit, moments to 1e-12)."""
    cases = []
    for s in (1.5, 1.9):
        for eps in (1e-2, 1e-3, 1e-4):
            for seed in range(85):
                cases.append(W.burgers(seed, jmax=14, eps=eps, s=s))
    announce("bench whole run", len(cases))
    ps, ms = [c[0] for c in cases], [c[1] for c in cases]
    b = mrlbm.Batch(ps, ms)
    try:
        b.set_block(512)
        b.set_capacity(999)
        b.set_schedule(256)
        nsteps = 3277
        b.step(nsteps)
        picked = []
        for eps in (1e-2, 1e-3, 1e-4):
            idx = [i for i, p in enumerate(ps) if p["eps"] == eps and p["s"][0] == 1.9]
            picked.append(max(idx, key=lambda i: b.stats(i)["tree_cells"]))
        for i in picked:
            announce("whole-run instance", i, "tree cells", b.stats(i)["tree_cells"])
            ora = make_oracle(ps[i], ms[i]).step(nsteps)
            lv, ix = b.leaves(i)
            olv, oix = ora.leaf_list()
            assert np.array_equal(lv, olv) and np.array_equal(ix, oix), i
            assert rel_err(b.moments(i), ora.leaf_conserved()) <= 1e-12, i
            assert b.stats(i)["leaf_updates"] == ora.leaf_updates, i
    finally:
        b.close()


def test_table2_column_I_configuration():
    """The configuration of the paper's Table 2, column I (D1Q2 advection of exp(-20 x^2) on
    [-3, 3], clamp boundaries, J = 9, eps = 1e-4, mu_bar = 30) through the C ABI: leaf set
    bit-exact with the oracle at the final step, and the ratio E / delta equal to the
    oracle's at every relaxation rate of the table."""
    import math
    W9, XMIN, XMAX = 9, -3.0, 3.0
    width = 1.0 / math.sqrt(20.0)
    e = W.edges(W9, XMIN, XMAX)
    u0 = W.avg_gauss_periodic(e, 1.0, 0.0, width, period=XMAX - XMIN, images=(0,))
    n_steps = W.n_steps(0.4, 1.0, W9, XMIN, XMAX)
    t = n_steps * (XMAX - XMIN) / 2 ** W9
    exact = W.avg_gauss_periodic(e, 1.0, 0.75 * t, width, period=XMAX - XMIN, images=(0,))
    for s in (0.75, 1.0, 1.25, 1.5, 1.75):
        p = W.base_params(scheme=W.D1Q2, physics=W.ADVECTION, lam=1.0, s=[s], phys=[0.75, 1.0, 1.4, 0.9],
                          jmin=2, jmax=W9, eps=1e-4, mu_bar=30, bc=W.CLAMP, x_min=XMIN, x_max=XMAX)
        announce("table 2 column I", "s", s)
        run = mrlbm.MRLBM(p, u0[None, :])
        run.step(n_steps)
        ora = make_oracle(p, u0[None, :]).step(n_steps)
        lv, ix = run.leaves()
        olv, oix = ora.leaf_list()
        assert np.array_equal(lv, olv) and np.array_equal(ix, oix)
        ref = UniformLBM(scheme_from_params(p), W9, W.CLAMP, u0[None, :]).step(n_steps)
        E = metrics.delta(exact[None, :], ref.conserved(), XMIN, XMAX)[0]
        d_gpu = metrics.delta(ref.conserved(), run.moments(mrlbm.FINEST), XMIN, XMAX)[0]
        d_ora = metrics.delta(ref.conserved(), ora.finest_conserved(), XMIN, XMAX)[0]
        assert abs(E / d_gpu - E / d_ora) <= 1e-9 * (E / d_ora), (s, E / d_gpu, E / d_ora)
        run.close()


# ------------------------------------------------------------------ reconstructed collision
@pytest.mark.parametrize("kind", KINDS)
def test_reconstructed_collision_parity(kind):
    """Reconstructed collision (Sec. 4.3.1, eq. reconstructedCollision) through the C ABI
    against the oracle's: leaf sets bit-exact and moments within 1e-12 every 15 steps, with
    leaves down to J_min = 2 (up to 2^7 finest cells reconstructed per leaf)."""
    p, mc = W.small_case(kind, seed=3, jmax=9, eps=1e-3)
    run_pair(dict(p, collision="reconstructed"), mc, 60, 15, f"recon {kind}")
    if kind == "burgers_d1q2":
        # the flag reaches the kernel: on a nonlinear flux the two collisions differ
        a, b = mrlbm.MRLBM(dict(p, collision="reconstructed"), mc), mrlbm.MRLBM(p, mc)
        a.step(30)
        b.step(30)
        assert not np.array_equal(a.moments(mrlbm.FINEST), b.moments(mrlbm.FINEST))
        a.close()
        b.close()


def test_reconstructed_collision_hbm_path_and_mixed_batch():
    """Runs with the reconstructed collision next to runs with the leaves collision in one
    batch (one kernel serves both), on chip and with every tree in HBM (capacity 0): each run
    equals its oracle bit for bit in its leaf set."""
    ps, ms = [], []
    for i, kind in enumerate(["burgers_d1q2", "advection", "burgers_d1q2"]):
        p, mc = W.small_case(kind, seed=10 + i, jmax=8, eps=1e-3)
        ps.append(dict(p, collision="reconstructed" if i != 1 else "leaves"))
        ms.append(mc)
    for cap in (-1, 0):
        announce("recon mixed batch", "capacity", cap)
        b = mrlbm.Batch(ps, ms)
        if cap >= 0:
            b.set_capacity(cap)
        b.step(20)
        b.step(20)
        for i, (p, mc) in enumerate(zip(ps, ms)):
            ora = make_oracle(p, mc).step(40)
            lv, ix = b.leaves(i)
            olv, oix = ora.leaf_list()
            assert np.array_equal(lv, olv) and np.array_equal(ix, oix), (cap, i)
            assert rel_err(b.moments(i), ora.leaf_conserved()) <= 1e-12, (cap, i)
        b.close()


def test_reconstructed_collision_fp32_within_bound():
    """FP32 storage with the reconstructed collision: within 1e-5 relative plus the eps bound
    of the FP64 oracle run."""
    p, mc = W.small_case("burgers_d1q2", seed=5, jmax=9, eps=1e-4)
    p = dict(p, collision="reconstructed")
    announce("recon fp32")
    n = 60
    run = mrlbm.MRLBM(dict(p, precision=mrlbm.FP32_STORAGE), mc)
    run.step(n)
    ora = make_oracle(p, mc).step(n)
    ref = UniformLBM(scheme_from_params(p), p["jmax"], p["bc"], mc).step(n)
    m32 = run.moments(mrlbm.FINEST)
    m64 = ora.finest_conserved()
    d64 = metrics.delta(ref.conserved(), m64, p["x_min"], p["x_max"])
    d3264 = metrics.delta(m64, m32, p["x_min"], p["x_max"])
    norm = metrics.delta(np.zeros_like(m64), m64, p["x_min"], p["x_max"])
    for c in range(m64.shape[0]):
        assert d3264[c] <= 1e-5 * norm[c] + 2.0 * max(d64[c], p["eps"]), (c, d3264, d64)
    run.close()


def test_reconstructed_collision_refuses_the_predictor():
    """The refinement predictor runs with the leaves collision only."""
    p, mc = W.small_case("burgers_d1q2", seed=1, jmax=8, eps=1e-3)
    run = mrlbm.MRLBM(dict(p, collision="reconstructed"), mc)
    with pytest.raises(mrlbm.MRLBMError):
        run.set_predictor(None, mrlbm.PRED_RECORD, sample_capacity=1000)
    run.step(3)
    assert run.stats()["steps"] == 3
    run.close()


def test_paper_test_V_through_the_c_abi():
    """The paper's Test V setup (Burgers, hat datum on [-1, 1], J = 9, mu_bar = 0, clamp,
    T = 1.3) through the C ABI: with the reconstructed collision the leaf set is bit-exact
    with the oracle's at every eps, and delta / eps stays below 1.5, while with the leaves
    collision it grows more than 10x from eps = 1e-2 to 1e-5, as on the oracle."""
    J, XMIN, XMAX = 9, -3.0, 3.0
    e = W.edges(J, XMIN, XMAX)
    dx = e[1] - e[0]
    xs = e[:-1, None] + (np.arange(256) + 0.5)[None, :] * dx / 256
    u0 = np.where(np.abs(xs) <= 1.0, 1.0 - np.abs(xs), 0.0).mean(1)
    n_steps = W.n_steps(1.3, 1.0, J, XMIN, XMAX)
    base = W.base_params(scheme=W.D1Q2, physics=W.BURGERS, lam=1.0, s=[1.25], jmin=2, jmax=J, mu_bar=0,
                         bc=W.CLAMP, x_min=XMIN, x_max=XMAX)
    ref = UniformLBM(scheme_from_params(base), J, W.CLAMP, u0[None, :]).step(n_steps).conserved()
    ratio = {}
    for coll in ("leaves", "reconstructed"):
        for eps in (1e-2, 1e-5):
            p = dict(base, eps=eps, collision=coll)
            announce("test V", coll, eps)
            run = mrlbm.MRLBM(p, u0[None, :])
            run.step(n_steps)
            if coll == "reconstructed":
                ora = make_oracle(p, u0[None, :]).step(n_steps)
                lv, ix = run.leaves()
                olv, oix = ora.leaf_list()
                assert np.array_equal(lv, olv) and np.array_equal(ix, oix), eps
            ratio[coll, eps] = metrics.delta(ref, run.moments(mrlbm.FINEST), XMIN, XMAX)[0] / eps
            run.close()
    assert ratio["leaves", 1e-5] / ratio["leaves", 1e-2] > 10.0, ratio
    assert max(ratio["reconstructed", 1e-2], ratio["reconstructed", 1e-5]) < 1.5, ratio


def test_euler_workload_against_the_exact_solution():
    """The Euler Riemann workload at full size through the C ABI, checked against the exact
    solution instead of the oracle: the reference scheme's error E (the library at eps = 0)
    falls from J = 12 to J = 14 by at least 2^0.8, the adaptive run's error e at eps = 1e-4 is
    within its perturbation delta of E, and delta stays below a tenth of E."""
    from oracle import exact
    GAM = 1.4
    out = {}
    for J in (12, 14):
        p, mc = W.euler(2, jmax=J, eps=1e-4)
        n = 60 * 2 ** (J - 9)
        t = n * (p["x_max"] - p["x_min"]) / 2 ** J / p["lam"]
        rl, rr = mc[0][0], mc[0][-1]
        ul, ur = mc[1][0] / rl, mc[1][-1] / rr
        pl = (GAM - 1.0) * (mc[2][0] - 0.5 * rl * ul * ul)
        pr = (GAM - 1.0) * (mc[2][-1] - 0.5 * rr * ur * ur)
        ex = exact.cell_averages(lambda xi: exact.euler_riemann(rl, ul, pl, rr, ur, pr, GAM, xi),
                                 p["x_min"], p["x_max"], J, 0.0, t)
        announce("euler exact", "J", J, "steps", n)
        ref = mrlbm.MRLBM(dict(p, eps=0.0), mc)
        ada = mrlbm.MRLBM(p, mc)
        ref.step(n)
        ada.step(n)
        mr, ma = ref.moments(mrlbm.FINEST), ada.moments(mrlbm.FINEST)
        E = metrics.delta(ex, mr, p["x_min"], p["x_max"])[0]
        e = metrics.delta(ex, ma, p["x_min"], p["x_max"])[0]
        d = metrics.delta(mr, ma, p["x_min"], p["x_max"])[0]
        out[J] = (E, e, d)
        print(f"[exact] J={J} steps={n} E={E:.4e} e={e:.4e} delta={d:.4e} E/delta={E / d:.1f} "
              f"leaves={ada.stats()['leaves']}", flush=True)
        ref.close()
        ada.close()
        assert abs(e - E) <= d * (1 + 1e-9), (J, E, e, d)
        assert d < 0.1 * E, (J, E, d)
    assert out[12][0] / out[14][0] > 2 ** 0.8, out


@pytest.mark.parametrize("seed", range(24))
def test_seeded_configuration_sweep(seed):
    """A seeded sweep over the parameters the other cases fix: family, gamma (1..3), J_min
    (1..3, with at least 2 gamma + 1 coarse cells on a periodic domain), J (6..9), eps
    (1e-2..1e-4), mu_bar (0..2) and the collision (reconstructed only with gamma = 1); leaf sets
    bit-exact with the oracle and moments within 1e-12 every 10 steps over 30 steps."""
    rng = np.random.default_rng([9, seed])
    kind = KINDS[int(rng.integers(len(KINDS)))]
    gamma = int(rng.integers(1, 4))
    jmax = int(rng.integers(6, 10))
    p, mc = W.small_case(kind, seed=int(rng.integers(1000)), jmax=jmax, eps=float(rng.choice([1e-2, 1e-3, 1e-4])))
    jmin = int(rng.integers(1, 4))
    if p["bc"] == W.PERIODIC:
        while 2 ** jmin < 2 * gamma + 1:
            jmin += 1
    coll = "reconstructed" if gamma == 1 and rng.random() < 0.5 else "leaves"
    p = dict(p, gamma=gamma, jmin=jmin, mu_bar=int(rng.integers(0, 3)), collision=coll)
    assert mrlbm.validate(p) == mrlbm.OK, p
    run_pair(p, mc, 30, 10, f"sweep {seed} {kind} gamma {gamma} J {jmin}..{jmax} {coll}")


def test_reconstructed_collision_at_full_size():
    """The reconstructed collision on the benchmark's D1Q3 Burgers workload at its full size
    (J = 14, leaves down to J_min = 2: up to 4096 finest cells per leaf), 60 steps from t = 0:
    leaf sets bit-exact and moments within 1e-12 every 20 steps."""
    p, mc = W.burgers(0, jmax=14, eps=1e-4, s=1.9)
    run_pair(dict(p, collision="reconstructed"), mc, 60, 20, "recon burgers J14")


@pytest.mark.parametrize("seed", range(12))
def test_seeded_fp32_sweep(seed):
    """FP32 storage over a seeded sweep of family, gamma, J_min, J, eps and collision: the
    finest-level moments after 30 steps within 1e-5 relative plus the eps bound of the FP64
    oracle run (details and thresholds stay FP64, so the trees may differ near thresholds)."""
    rng = np.random.default_rng([10, seed])
    kind = KINDS[int(rng.integers(len(KINDS)))]
    gamma = int(rng.integers(1, 4))
    jmax = int(rng.integers(6, 10))
    p, mc = W.small_case(kind, seed=int(rng.integers(1000)), jmax=jmax, eps=float(rng.choice([1e-3, 1e-4])))
    jmin = int(rng.integers(1, 4))
    if p["bc"] == W.PERIODIC:
        while 2 ** jmin < 2 * gamma + 1:
            jmin += 1
    coll = "reconstructed" if gamma == 1 and rng.random() < 0.5 else "leaves"
    p = dict(p, gamma=gamma, jmin=jmin, collision=coll)
    announce("fp32 sweep", seed, kind, "gamma", gamma, "J", jmin, jmax, coll)
    n = 30
    run = mrlbm.MRLBM(dict(p, precision=mrlbm.FP32_STORAGE), mc)
    run.step(n)
    ora = make_oracle(p, mc).step(n)
    ref = UniformLBM(scheme_from_params(p), p["jmax"], p["bc"], mc).step(n)
    m32 = run.moments(mrlbm.FINEST)
    m64 = ora.finest_conserved()
    d64 = metrics.delta(ref.conserved(), m64, p["x_min"], p["x_max"])
    d3264 = metrics.delta(m64, m32, p["x_min"], p["x_max"])
    norm = metrics.delta(np.zeros_like(m64), m64, p["x_min"], p["x_max"])
    for c in range(m64.shape[0]):
        assert d3264[c] <= 1e-5 * norm[c] + 2.0 * max(d64[c], p["eps"]), (c, d3264, d64)
    run.close()


@pytest.mark.parametrize("seed", range(4))
def test_seeded_batch_sweep(seed):
    """Heterogeneous batches: six D1Q2 runs (advection and Burgers) with J in 6..10, eps in
    1e-2..1e-4 and either collision in one launch, at a random block size and on-chip capacity
    (all trees in HBM, a small limit that moves trees between LDS and HBM, or the full LDS);
    every run bit-exact in its leaf set with its own oracle after 25 + 15 steps."""
    rng = np.random.default_rng([11, seed])
    ps, ms = [], []
    for i in range(6):
        kind = ["advection", "burgers_d1q2"][int(rng.integers(2))]
        p, mc = W.small_case(kind, seed=int(rng.integers(1000)), jmax=int(rng.integers(6, 11)),
                             eps=float(rng.choice([1e-2, 1e-3, 1e-4])))
        ps.append(dict(p, collision="reconstructed" if rng.random() < 0.5 else "leaves"))
        ms.append(mc)
    block = int(rng.choice([128, 256, 512]))
    cap = int(rng.choice([-1, 0, 200]))
    announce("batch sweep", seed, "block", block, "capacity", cap, [p["jmax"] for p in ps])
    b = mrlbm.Batch(ps, ms)
    b.set_block(block)
    b.set_capacity(cap)
    b.step(25)
    b.step(15)
    for i, (p, mc) in enumerate(zip(ps, ms)):
        ora = make_oracle(p, mc).step(40)
        lv, ix = b.leaves(i)
        olv, oix = ora.leaf_list()
        assert np.array_equal(lv, olv) and np.array_equal(ix, oix), (seed, i)
        assert rel_err(b.moments(i), ora.leaf_conserved()) <= 1e-12, (seed, i)
    b.close()
