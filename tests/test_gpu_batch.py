"""Batched form on the GPU: many matrices of uneven order in one persistent
launch must reproduce, bit for bit, the chains of each matrix swept alone by
the single-matrix path (same seed, stream_id = matrix index), and therefore
the oracle."""

import numpy as np
import pytest

import gen
import oracle
from gpu_util import oracle_matrix, print_case, rel_err

pytestmark = pytest.mark.gpu

mc = pytest.importorskip("paper_cs_0412107_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


SIZES = [200, 1500, 333, 2900, 64, 800, 1201, 450, 3000, 97, 640, 2048]


@pytest.fixture(scope="module")
def mats():
    return [gen.round_values(gen.pedigree(int(n), seed=300 + j), np.float32) for j, n in enumerate(SIZES)]


@pytest.mark.parametrize("schedule,noise", [(0, mc.MCINV_NOISE_NORMAL), (1, mc.MCINV_NOISE_NORMAL),
                                            (0, mc.MCINV_NOISE_RADEMACHER), (1, mc.MCINV_NOISE_RADEMACHER)])
def test_batched_states_equal_single_path(mats, schedule, noise):
    print_case(test="batch_states", matrices=len(mats), schedule=schedule, noise=noise)
    P, G, seed = 64, 16, 0x412107 + 3
    with mc.BatchSampler(mats, pairs=P, groups=G, seed=seed, rows_per_item=32, grab=2, schedule=schedule,
                         noise=noise) as b:
        b.burn_in(4)
        for m in (0, 3, 4, 9, 11):
            with mc.Sampler(mats[m], pairs=P, groups=G, dtype="f32", seed=seed, stream_id=m, noise=noise) as s:
                s.burn_in(4)
                for which in (0, 1):
                    assert np.array_equal(b.state(m, which), s.state(which)), (m, which)


def test_batched_hub_row_states_equal_single_path():
    """A merged row of ~2500 entries: the item holding it exceeds the entries
    staged in LDS per item and reads them from global memory, while the other
    items of the same launches are staged; both schedules must still give the
    single path's chains bit for bit."""
    from test_gpu_parity import _matrix
    hub = gen.round_values(_matrix("hub2500"), np.float32)
    mats = [gen.round_values(gen.pedigree(900, seed=701), np.float32), hub,
            gen.round_values(gen.pedigree(1700, seed=702), np.float32)]
    P, G, seed = 64, 16, 0x5151
    for schedule in (0, 1):
        print_case(test="batch_hub_states", schedule=schedule)
        with mc.BatchSampler(mats, pairs=P, groups=G, seed=seed, rows_per_item=16, grab=2, schedule=schedule) as b:
            b.burn_in(3)
            for m in range(len(mats)):
                with mc.Sampler(mats[m], pairs=P, groups=G, dtype="f32", seed=seed, stream_id=m) as s:
                    s.burn_in(3)
                    for which in (0, 1):
                        assert np.array_equal(b.state(m, which), s.state(which)), (schedule, m, which)


def test_batched_matches_oracle(mats):
    P, G, seed = 64, 16, 11
    m = 5
    ora = oracle.Run(mats[m], seed=seed, pairs=P, groups=G, stream=m)
    with mc.BatchSampler(mats, pairs=P, groups=G, seed=seed) as b:
        b.burn_in(3)
        ora.burn_in(3)
        assert rel_err(b.state(m, 0), ora.z) <= 1e-5
        assert rel_err(b.state(m, 1), ora.w) <= 1e-5


@pytest.mark.parametrize("P,G,schedule", [(64, 16, 0), (64, 16, 1), (32, 2, 0), (128, 8, 1)])
def test_batched_moments_equal_single_path(mats, P, G, schedule):
    print_case(test="batch_moments", P=P, G=G, schedule=schedule)
    seed, S, bd = 99, 12, 48
    with mc.BatchSampler(mats[:6], pairs=P, groups=G, seed=seed, rows_per_item=16, grab=1,
                         schedule=schedule) as b:
        b.burn_in(5)
        b.request(diag=True, block_dim=bd, expected_samples=S)
        b.sample(S)
        for m in (1, 3):
            with mc.Sampler(mats[m], pairs=P, groups=G, dtype="f32", seed=seed, stream_id=m) as s:
                s.burn_in(5)
                s.request(diag=True, trace=False)
                s.sample(S)
                d, se = s.diag()
            bd_, bse = b.diag(m)
            np.testing.assert_allclose(bd_, d, rtol=1e-12, atol=0)
            if G >= 16:
                np.testing.assert_allclose(bse, se, rtol=1e-9)
            # block: the single path with one group and bf16x3 products is the same MFMA sequence
            n = mats[m].n
            rows = np.arange(n - bd, n)
            with mc.Sampler(mats[m], pairs=P, groups=1, dtype="f32", seed=seed, stream_id=m,
                            moments="bf16x3") as s1:
                s1.burn_in(5)
                s1.request(diag=False, trace=False, block_rows=rows, block_cols=rows)
                s1.sample(S)
                sb, _ = s1.block()
            bb, bbse = b.block(m)
            np.testing.assert_allclose(bb, sb, rtol=1e-12, atol=1e-15)
            assert np.all(np.isfinite(bbse))
    # and the block against the fp64 oracle
    m = 3
    ora = oracle.Run(mats[m], seed=seed, pairs=P, groups=1, stream=m)
    ora.burn_in(5)
    n = mats[m].n
    rows = np.arange(n - bd, n)
    ora.request(S, diag=False, block_rows=rows, block_cols=rows, trace=False)
    ora.sample(S)
    ob, _ = ora.block()
    assert rel_err(bb, ob.real) <= 1e-4


@pytest.mark.parametrize("schedule", [0, 1])
def test_graph_replays_continue_the_chain(mats, schedule):
    """Three replays of a 3-sweep call equal one 9-sweep call."""
    P, G, seed = 64, 16, 5
    sub = mats[:5]
    with mc.BatchSampler(sub, pairs=P, groups=G, seed=seed, schedule=schedule) as a, \
            mc.BatchSampler(sub, pairs=P, groups=G, seed=seed, schedule=schedule) as b:
        a.burn_in(2)
        b.burn_in(2)
        a.request(diag=True, block_dim=32, expected_samples=9)
        b.request(diag=True, block_dim=32, expected_samples=9)
        for _ in range(3):
            a.sample(3)
        b.sample(9)
        for m in range(len(sub)):
            assert np.array_equal(a.state(m, 0), b.state(m, 0))
            da, _ = a.diag(m)
            db, _ = b.diag(m)
            assert np.array_equal(da, db)
        assert a.info()["samples_done"] == 9


def test_autotune_and_sample_until(mats):
    P, G, seed = 64, 16, 21
    with mc.BatchSampler(mats, pairs=P, groups=G, seed=seed) as b:
        sched, r, g, ms = b.autotune(1)
        assert sched in (0, 1) and r in (16, 32, 64, 128, 256, 512, 1024) and g in (1, 4) and ms > 0
        info = b.info()
        burned = info["sweeps_done"]
        b.burn_in(30)
        b.request(diag=True)
        done, ach = b.sample_until(0.05, 400, 10)
        assert ach <= 0.05 and done <= 400
        # the schedule does not change the chain: same state as the single path
        with mc.Sampler(mats[2], pairs=P, groups=G, dtype="f32", seed=seed, stream_id=2) as s:
            s.burn_in(burned + 30 + done)
            assert np.array_equal(b.state(2, 0), s.state(0))


@pytest.mark.parametrize("schedule", [0, 1])
def test_per_matrix_stop_equals_single_path(mats, schedule):
    """sample_until_each: every matrix stops at the first check where its own
    max SE/|est| meets the tolerance, exactly where the single path's
    sample_until stops it (same burn-in, seed and stream), with bit-identical
    chains and estimates; stopped matrices are frozen while the rest go on, and
    a new request makes every matrix active again."""
    print_case(test="batch_each", schedule=schedule)
    P, G, seed, rel, burn, bd = 64, 16, 77, 0.04, 20, 16
    sub = mats[:6]
    with mc.BatchSampler(sub, pairs=P, groups=G, seed=seed, schedule=schedule) as b:
        b.burn_in(burn)
        b.request(diag=True, block_dim=bd, expected_samples=400)
        done, ach = b.sample_until_each(rel, 2000, 10)
        samples, active = b.matrix_samples()
        assert not active.any() and ach <= rel
        assert done == samples.max() and len(set(samples.tolist())) >= 2, samples
        for m in range(len(sub)):
            with mc.Sampler(sub[m], pairs=P, groups=G, dtype="f32", seed=seed, stream_id=m) as s:
                s.burn_in(burn)
                s.request(diag=True, trace=False)
                dj, aj = s.sample_until(rel, 2000, 10)
                assert dj == samples[m], (m, dj, samples[m])
                d, se = s.diag()
                assert np.array_equal(b.state(m, 0), s.state(0))
                assert np.array_equal(b.state(m, 1), s.state(1))
            bd_, bse = b.diag(m)
            np.testing.assert_allclose(bd_, d, rtol=1e-12, atol=0)
            np.testing.assert_allclose(bse, se, rtol=1e-9)
        # block moments of the first matrix to stop: its own sample count
        m = int(np.argmin(samples))
        n = sub[m].n
        rows = np.arange(n - bd, n)
        with mc.Sampler(sub[m], pairs=P, groups=1, dtype="f32", seed=seed, stream_id=m, moments="bf16x3") as s1:
            s1.burn_in(burn)
            s1.request(diag=False, trace=False, block_rows=rows, block_cols=rows)
            s1.sample(int(samples[m]))
            sb, _ = s1.block()
        bb, _ = b.block(m)
        np.testing.assert_allclose(bb, sb, rtol=1e-12, atol=1e-15)
        # every matrix active again after a new request
        b.request(diag=True)
        samples2, active2 = b.matrix_samples()
        assert active2.all() and not samples2.any()
        b.sample(2)
        assert b.matrix_samples()[0].tolist() == [2] * len(sub)


def test_batch_errors(mats):
    with pytest.raises(mc.McinvError) as ei:
        mc.mcinv_batch_create(2, n_pairs=48)
    assert ei.value.code == mc.MCINV_EINVAL
    b = mc.mcinv_batch_create(2, n_pairs=64, n_groups=16)
    try:
        m = mats[0]
        mc.mcinv_batch_load_csr(b, 0, m.n, m.nnz, m.row_ptr, m.col, m.val)
        with pytest.raises(mc.McinvError) as ei:
            mc.mcinv_batch_burn_in(b, 1)
        assert ei.value.code == mc.MCINV_ESTATE
    finally:
        mc.mcinv_batch_destroy(b)
    with mc.BatchSampler(mats[:3], pairs=64, groups=16) as bs:
        with pytest.raises(mc.McinvError) as ei:
            bs.request(diag=True, block_dim=129)
        assert ei.value.code == mc.MCINV_EINVAL


@pytest.mark.parametrize("schedule", [0, 1])
def test_batched_coupled_burn_in_equals_single_path(mats, schedule):
    """The batch burns in for the largest of the matrices' own coupling
    lengths (the difference iteration is the single path's, bit for bit), and
    every matrix's chains then equal the single path after that many sweeps."""
    print_case(test="batch_coupled", schedule=schedule)
    P, G, seed, tol = 64, 16, 31, 5e-5
    sub = mats[:6]
    Ns = []
    for j, x in enumerate(sub):
        with mc.Sampler(x, pairs=P, groups=G, dtype="f32", seed=seed, stream_id=j) as s:
            n, dz, dw = s.burn_in_coupled(tol, 500)
            Ns.append(n)
    with mc.BatchSampler(sub, pairs=P, groups=G, seed=seed, schedule=schedule) as b:
        N, worst = b.burn_in_coupled(tol, 500)
        assert N == max(Ns) and worst < tol
        for j in (0, 2, 5):
            with mc.Sampler(sub[j], pairs=P, groups=G, dtype="f32", seed=seed, stream_id=j) as s:
                s.burn_in(N)
                assert np.array_equal(b.state(j, 0), s.state(0))
                assert np.array_equal(b.state(j, 1), s.state(1))


def test_batched_full_size_sampled_pairs():
    """The batched workload in the benchmark's launch configuration (512
    pedigree matrices, n log-uniform in [1e3, 5e4], 64 pairs, autotuned
    schedule): sampled pair columns of three matrices against the oracle."""
    w = gen.WORKLOADS["batched"]
    big = [gen.round_values(x, np.float32) for x in gen.batched_pedigrees(w["m"], w["lo"], w["hi"], w["seed"])]
    P, G, seed = w["pairs"], w["groups"], w["noise_seed"]
    print_case(test="batch_full", matrices=len(big), rows=sum(x.n for x in big))
    with mc.BatchSampler(big, pairs=P, groups=G, seed=seed) as b:
        b.autotune(1)
        b.burn_in(2)
        k = b.info()["sweeps_done"]
        pids = np.array([0, 5, 63])
        for m in (0, 255, 511):
            ora = oracle.Run(big[m], seed=seed, pairs=P, pair_ids=pids, stream=m)
            ora.burn_in(k)
            assert rel_err(b.state(m, 0)[:, pids], ora.z) <= 1e-5
            assert rel_err(b.state(m, 1)[:, pids], ora.w) <= 1e-5


def test_stop_rule_needs_long_time_batches(mats):
    """With fewer than 16 chain groups the diagonal's error clusters are time
    batches of ceil(expected_samples / 16) sweeps: both stopping rules refuse
    batches shorter than 16 sweeps (their SE would run small), and with long
    enough batches the stopped estimates lie within their errors of the exact
    inverse."""
    print_case(test="batch_stop_batches")
    sub = [mats[0], mats[4], mats[9]]
    P, G, seed = 64, 4, 31
    with mc.BatchSampler(sub, pairs=P, groups=G, seed=seed) as b:
        b.burn_in(40)
        b.request(diag=True, expected_samples=100)   # batches of 7 sweeps
        for call in (b.sample_until, b.sample_until_each):
            with pytest.raises(mc.McinvError) as ei:
                call(0.05, 400, 10)
            assert ei.value.code == mc.MCINV_EINVAL
        b.request(diag=True, expected_samples=640)   # batches of 40 sweeps
        done, ach = b.sample_until_each(0.02, 4000, 20)
        samples, active = b.matrix_samples()
        assert not active.any() and ach <= 0.02
        assert samples.min() >= 16 * 2   # at least two time batches per matrix
        z = []
        for m, mat in enumerate(sub):
            exact = np.diag(np.linalg.inv(gen.to_dense(mat)))
            d, se = b.diag(m)
            z.append((d - exact) / se)
        z = np.concatenate(z)
        assert np.max(np.abs(z)) < 4.5
        assert 0.5 <= np.mean(z ** 2) <= 1.6


def test_surrogate_labels_against_oracle(mats):
    """mcinv_batch_read_labels: the surrogate's training targets c_ii (C^-1)_ii
    and their errors |c_ii| SE_i, formed in the library from the batched
    diagonal estimates, against the oracle's estimates of the same chains
    (same seed, stream_id = matrix index, all 64 pairs) scaled by c_ii here."""
    print_case(test="batch_labels")
    sub = [mats[0], mats[4], mats[9]]
    P, G, seed, burn, S = 64, 16, 55, 20, 40
    with mc.BatchSampler(sub, pairs=P, groups=G, seed=seed) as b:
        b.burn_in(burn)
        b.request(diag=True, expected_samples=S)
        b.sample(S)
        for j, m in enumerate(sub):
            y, y_se = b.labels(j)
            ora = oracle.Run(m, seed=seed, pairs=P, groups=G, stream=j)
            ora.burn_in(burn)
            ora.request(S, diag=True, trace=False)
            ora.sample(S)
            est, se = ora.diag()
            rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
            on = np.asarray(m.col) == rows
            cii = np.zeros(m.n)
            cii[rows[on]] = np.asarray(m.val)[on]
            np.testing.assert_allclose(y, cii * est.real, rtol=2e-5, atol=0)
            np.testing.assert_allclose(y_se, np.abs(cii) * se, rtol=2e-4, atol=0)
            # and the library's own estimates, scaled: the same numbers bit for bit
            d, dse = b.diag(j)
            assert np.array_equal(y, cii * d) and np.array_equal(y_se, np.abs(cii) * dse)
