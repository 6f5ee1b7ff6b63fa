"""Batched ensembles: every box of a batch evolves bit for bit as the same
box in a single-grid handle (same per-box CFL step, same tile arithmetic),
whatever the launch shape, eagerly or replayed from a captured HIP graph."""
import sys

import numpy as np
import pytest

from paper_1004_1680_amd import inputs as I

pytestmark = pytest.mark.gpu

DIMS = [(16, 16, 16), (24, 16, 32), (32, 32, 32), (8, 12, 16), (48, 48, 48)]


@pytest.fixture(scope="module")
def M():
    from paper_1004_1680_amd import mhd
    mhd.load()
    return mhd


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def states(dims):
    return [I.random_smooth(n, seed=40 + i) for i, n in enumerate(dims)]


def single_runs(M, dims, ss, prec, nsteps):
    out, times = [], []
    for n, s in zip(dims, ss):
        S = M.Solver(n, prec=prec)
        S.set_state(s)
        for _ in range(nsteps):
            S.step_auto(0.7)
        assert S.status() == nsteps
        out.append(S.get_state())
        times.append(S.time())
        S.close()
    return out, times


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_single_boxes(M, prec, graph):
    say(f"case: batch vs single, {prec}, graph={graph}")
    ss = states(DIMS)
    ref, rtimes = single_runs(M, DIMS, ss, prec, 3)
    B = M.Batch(DIMS, prec=prec)
    for i, s in enumerate(ss):
        B.set_state(i, s)
    B.run(3, graph=graph)
    steps, nonphys = B.status()
    assert list(steps) == [3] * len(DIMS) and not nonphys.any()
    for i in range(len(DIMS)):
        assert np.array_equal(B.get_state(i), ref[i]), i
    assert np.array_equal(B.times(), np.array(rtimes))
    B.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_reverse_pairs_fused_or_separate(M, prec):
    """the batch runs each reverse-half pair M_d F_d in one launch or as two
    operators; either way every box equals its single-grid run, which uses
    the tier's other default (fused in FP32, separate in FP64)"""
    say(f"case: batch reverse pairs, {prec}")
    ss = states(DIMS)
    ref, _ = single_runs(M, DIMS, ss, prec, 2)
    B = M.Batch(DIMS, prec=prec)
    other = 2 if prec == "f32" else 1
    B.set_launch(M.MHD_BATCH_REVERSE, other)
    assert B.launch(M.MHD_BATCH_REVERSE) == other
    # fused pairs with chunks of their own (8: the shortest, below the warm-up)
    B.set_launch(M.MHD_BATCH_PAIR_CHUNK, 8)
    assert B.launch(M.MHD_BATCH_PAIR_CHUNK) == 8
    for i, s in enumerate(ss):
        B.set_state(i, s)
    B.run(2, graph=True)
    B.status()
    for i in range(len(DIMS)):
        assert np.array_equal(B.get_state(i), ref[i]), i
    B.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_middle_in_one_launch(M, graph):
    """the middle of a step M_z M_z F_z as one launch over the pairs' work
    list: every box equals its single-grid run (which at these sizes runs M_z
    and the z pair), with the shortest and a longer pair chunk"""
    say(f"case: batch middle in one launch, graph={graph}")
    ss = states(DIMS)
    ref, rtimes = single_runs(M, DIMS, ss, "f32", 3)
    for pchunk in (8, 32):
        B = M.Batch(DIMS, prec="f32")
        assert B.launch(M.MHD_BATCH_MIDDLE) == 2          # built in: boxes below 128^3 on average
        B.set_launch(M.MHD_BATCH_MIDDLE, 1)
        assert B.launch(M.MHD_BATCH_MIDDLE) == 1
        B.set_launch(M.MHD_BATCH_PAIR_CHUNK, pchunk)
        for i, s in enumerate(ss):
            B.set_state(i, s)
        B.run(3, graph=graph)
        steps, nonphys = B.status()
        assert list(steps) == [3] * len(DIMS) and not nonphys.any()
        for i in range(len(DIMS)):
            assert np.array_equal(B.get_state(i), ref[i]), (pchunk, i)
        assert np.array_equal(B.times(), np.array(rtimes))
        B.close()
    T = M.Batch(DIMS, prec="f64")
    T.set_launch(M.MHD_BATCH_MIDDLE, 1)
    assert T.launch(M.MHD_BATCH_MIDDLE) == 2              # FP32 only
    T.close()


def test_batch_middle_odd_step_counts(M):
    """with the fused middle the face fields change buffer every step and the
    captured graph holds two steps: runs of 1, 2 and 3 steps in turn (eager
    steps realign the buffers around graph replays) and a state set between
    them all match single grids"""
    say("case: batch middle, odd step counts")
    ss = states(DIMS)
    ref, rtimes = single_runs(M, DIMS, ss, "f32", 6)
    B = M.Batch(DIMS, prec="f32")
    B.set_launch(M.MHD_BATCH_MIDDLE, 1)
    for i, s in enumerate(ss):
        B.set_state(i, s)
    B.run(1, graph=True)
    B.run(2, graph=True)
    B.run(3, graph=True)
    steps, nonphys = B.status()
    assert list(steps) == [6] * len(DIMS) and not nonphys.any()
    for i in range(len(DIMS)):
        assert np.array_equal(B.get_state(i), ref[i]), i
    assert np.array_equal(B.times(), np.array(rtimes))
    # a box set afresh at an odd buffer phase starts from its new state
    ref1, _ = single_runs(M, DIMS[:1], ss[:1], "f32", 1)
    B.run(1, graph=True)
    B.set_state(0, ss[0])
    B.run(1, graph=True)
    assert np.array_equal(B.get_state(0), ref1[0])
    B.close()


@pytest.mark.parametrize("grid,chunk,pchunk", [(8, 8, 256), (64, 16, 8), (1024, 64, 128), (2048, 256, 32)])
def test_batch_launch_shape_invariance(M, grid, chunk, pchunk):
    say(f"case: batch launch grid={grid} chunk={chunk} pair chunk={pchunk}")
    ss = states(DIMS)
    ref, _ = single_runs(M, DIMS, ss, "f32", 2)
    B = M.Batch(DIMS, prec="f32")
    for key in (M.MHD_BATCH_GRID_X, M.MHD_BATCH_GRID_Y, M.MHD_BATCH_GRID_Z):
        B.set_launch(key, grid)
    B.set_launch(M.MHD_BATCH_CHUNK, chunk)
    B.set_launch(M.MHD_BATCH_PAIR_CHUNK, pchunk)
    for i, s in enumerate(ss):
        B.set_state(i, s)
    B.run(2, graph=True)
    B.status()
    for i in range(len(DIMS)):
        assert np.array_equal(B.get_state(i), ref[i]), i


def test_graph_replays_interleaved_with_eager_work(M):
    # each replay of the captured step is checked against eager steps, with
    # host synchronisation and eager kernels of another handle in between
    say("case: graph replays vs eager")
    ss = states(DIMS[:3])
    G = M.Batch(DIMS[:3], prec="f32")
    E = M.Batch(DIMS[:3], prec="f32")
    for i, s in enumerate(ss):
        G.set_state(i, s)
        E.set_state(i, s)
    for rep in range(4):
        G.run(1, graph=True)
        E.run(1, graph=False)
        G.status()
        E.status()
        for i in range(3):
            assert np.array_equal(G.get_state(i), E.get_state(i)), (rep, i)
        assert np.array_equal(G.times(), E.times())


def test_nonphysical_box_is_isolated(M):
    say("case: non-physical box in a batch")
    dims = DIMS[:3]
    ss = states(dims)
    bad = I.uniform(dims[1])
    bad[4, 2, 3, 4] = 0.1                      # negative pressure in one cell
    ss[1] = bad
    B = M.Batch(dims, prec="f32")
    for i, s in enumerate(ss):
        B.set_state(i, s)
    B.run(2, graph=True)
    steps, nonphys = B.status(raise_on_nonphysical=False)
    assert list(nonphys) == [0, 1, 0]
    assert steps[0] == 2 and steps[1] == 0 and steps[2] == 2
    good, _ = single_runs(M, [dims[0], dims[2]], [ss[0], ss[2]], "f32", 2)
    assert np.array_equal(B.get_state(0), good[0])
    assert np.array_equal(B.get_state(2), good[1])
    assert np.array_equal(B.get_state(1), bad.astype(np.float32).astype(np.float64))


def test_ensemble_family_sampled_boxes(M):
    # the uneven-ensemble generator (per-box Mach in [0.5, 3], beta in
    # [0.1, 10]) on small sizes; three sampled boxes against single runs
    say("case: ensemble family, sampled boxes")
    spec = I.ensemble_spec(nbox=12, seed=4, sizes=(32, 48))
    dims = [(n, n, n) for n, _, _, _ in spec]
    ss = [I.turbulence((n, n, n), seed=sd, mach=m, beta=b) for n, m, b, sd in spec]
    B = M.Batch(dims, prec="f32")
    for i, s in enumerate(ss):
        B.set_state(i, s)
    B.run(3, graph=True)
    steps, nonphys = B.status(raise_on_nonphysical=False)
    checked = 0
    for i in range(len(dims)):
        if nonphys[i]:        # a Mach-3 box may leave the physical range: the
            continue          # method has no floors; compare the others
        if checked == 3:
            break
        ref, _ = single_runs(M, [dims[i]], [ss[i]], "f32", 3)
        assert np.array_equal(B.get_state(i), ref[0]), i
        checked += 1
    assert checked == 3


def test_batch_rejects_bad_arguments(M):
    with pytest.raises(M.MHDError):
        M.Batch([(16, 16, 16), (10, 16, 16)])
    B = M.Batch([(16, 16, 16)])
    with pytest.raises(M.MHDError):
        B.set_launch(M.MHD_BATCH_GRID_X, 12)
    with pytest.raises(M.MHDError):
        B.set_launch(99, 8)
    with pytest.raises(ValueError):
        B.set_state(0, np.zeros((8, 8, 8, 8)))


def test_benchmark_ensemble_sampled_boxes(M):
    """the benchmark's ensemble (64 boxes of {32..256}^3, 312 M cells) in its
    launch configuration (persistent launches, graph replay): sampled boxes
    (the smallest, the largest, one in between) equal single-grid handles
    of the same box bit for bit after two steps"""
    from paper_1004_1680_amd import inputs as I
    say("case: benchmark ensemble, sampled boxes")
    spec = I.ensemble_spec(nbox=64, seed=4)
    dims = [(n, n, n) for n, _, _, _ in spec]
    B = M.Batch(dims, prec="f32")
    keep = {}
    sizes = [n for n, _, _, _ in spec]
    picks = {sizes.index(min(sizes)), sizes.index(max(sizes)), len(spec) // 2}
    for i, (n, m, b, sd) in enumerate(spec):
        s = I.turbulence((n, n, n), seed=sd, mach=m, beta=b)
        B.set_state(i, s)
        if i in picks:
            keep[i] = s
    say("boxes resident; cells", B.ncell)
    B.run(2, graph=True)
    steps, nonphys = B.status(raise_on_nonphysical=False)
    for i, s in keep.items():
        n = dims[i]
        S = M.Solver(n, prec="f32")
        S.set_state(s)
        say("box", i, n, "steps", int(steps[i]), "record", int(nonphys[i]))
        if nonphys[i]:
            with pytest.raises(M.NonPhysicalState):   # the single grid stops too
                S.run(2)
        else:
            S.run(2)
            assert steps[i] == 2
            assert np.array_equal(B.get_state(i), S.get_state()), i
        S.close()
    B.close()
