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
