"""The trained closure against the plain coarse solver (GPU, end to end).

Training pairs come from 256^3 fine runs of seeded Orszag-Tang-type states
restricted by 8 to 32^3 (fine solver, restriction, residual and statistics
kernels); the network is trained by the library's MFMA forward/backward
kernels and Adam, then a held-out state is rolled out 24 learned coarse
steps.  The learned 32^3 solution must be closer to the restricted fine
solution (relative L1 over the 8 fields) than the plain 32^3 solution at
the same time, and the plain 64^3 solution (restricted to 32^3) must be
closer still than the plain 32^3 one (the error measure is sound)."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_learned_closure_beats_the_plain_coarse_solver():
    from paper_1004_1680_amd import closure_train as CT
    print("case: closure training 256^3 -> 32^3, 12 trajectories x 24 steps", flush=True)
    res, cl = CT.run(nf=256, r=8, train_seeds=tuple(range(1, 13)), steps_per_traj=24, epochs=10,
                     eval_steps=24, log=lambda m: (print(m), sys.stdout.flush()))
    L, p32, p64 = res["learned"]["L1"], res["plain_32"]["L1"], res["plain_64"]["L1"]
    print(f"L1 learned {L:.4e}, plain 32^3 {p32:.4e}, plain 64^3 {p64:.4e}", flush=True)
    assert p64 < p32
    assert L < 0.9 * p32
    assert res["history"][-1][1] < res["val_loss_untrained"]
    cl.close()


def test_training_continues_from_saved_weights(tmp_path):
    """a second run over new seeds starts from the saved parameters, keeps
    the saved scales and gate, and counts the pairs of both runs"""
    import time

    import numpy as np

    from paper_1004_1680_amd import closure_train as CT
    print("case: closure training continued from saved weights, 256^3 -> 32^3", flush=True)
    log = lambda m: (print(m), sys.stdout.flush())
    cl, scales, info = CT.train_closure(nf=256, r=8, train_seeds=(1, 2), steps_per_traj=3, val_steps=2,
                                        epochs=2, log=log, weighting="sqrt", gate=True)
    path = str(tmp_path / "first.npz")
    CT.save(path, cl, scales, info, info["gate"])
    p1 = cl.params().copy()
    cl.close()
    cl2, scales2, info2 = CT.train_closure(nf=256, r=8, train_seeds=(3,), steps_per_traj=3, val_steps=2,
                                           epochs=2, log=log, weighting="sqrt", gate=True, init=path)
    assert info["pairs"] == 6 and info2["pairs"] == 3
    assert info2["pairs_total"] == 9
    assert [r["pairs"] for r in info2["runs"]] == [6, 3]
    assert [r["seeds"] for r in info2["runs"]] == [[1, 2], [3]]
    for a, b in zip(scales, scales2):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    assert info2["gate"] == info["gate"]
    p2 = cl2.params()
    assert np.all(np.isfinite(p2)) and not np.array_equal(p1, p2)
    # a deadline already past generates nothing
    import torch
    none = CT.generate_pairs(cl2, 256, 8, (4,), 3, torch.cuda.current_stream(), log=log,
                             deadline=time.perf_counter())
    assert len(none) == 0
    cl2.close()
