"""Shared comparison of per-rotation GPU results with the FP64 oracle (not a test module).

Bar: validity identical; |score_gpu - score_oracle| <= 1e-4; the per-rotation displacement is
identical unless the oracle's best and runner-up on that rotation are within 2e-4 (then the
GPU's displacement must score within 2e-4 of the oracle's best on the oracle's map); N at the
GPU's displacement exact; the overall best rotation identical unless the oracle's two best
rotations are within 2e-4 (then the GPU's pick must score within 2e-4 of the best).
"""
import numpy as np

import oracle as O

CTOL = 1e-4
TIE = 2e-4


def check_against_oracle(A, B, rotations, per, best, P=None, gamma=0.5, measure="squared", mask_b=None,
                         mask_a=None):
    """Run the oracle on every rotation and check the GPU's per-rotation results and best."""
    A = np.asarray(A)
    B = np.asarray(B)
    res, ob = O.evaluate(A, B, rotations, mask_a=mask_a, mask_b=mask_b, gamma=gamma, P_xyz=P, keep_maps=True,
                         measure=measure)
    nza, nya, nxa = A.shape
    for i, (g, r) in enumerate(zip(per, res)):
        assert bool(g.valid) == bool(r.valid), (i, g.valid, r.valid)
        if not r.valid:
            continue
        assert abs(float(g.score) - r.score) <= CTOL, (i, float(g.score), r.score)
        C = r.C
        v = np.isfinite(C)
        top = np.partition(C[v], -2)[-2:] if v.sum() > 1 else None
        iz, iy, ix = g.shift[2] + nza - 1, g.shift[1] + nya - 1, g.shift[0] + nxa - 1
        if top is None or top[1] - top[0] >= TIE:
            assert tuple(g.shift) == r.shift, (i, tuple(g.shift), r.shift)
        else:
            assert C[iz, iy, ix] >= r.score - TIE, (i, tuple(g.shift), r.shift)
        assert g.overlap == r.N[iz, iy, ix], (i, g.overlap, int(r.N[iz, iy, ix]))
    if ob is None:
        assert best.rot_index == -1
        return res, ob
    scores = np.array([r.score for r in res])
    order = np.sort(scores[np.isfinite(scores)])[::-1]
    if order.size < 2 or order[0] - order[1] >= TIE:
        assert best.rot_index == ob, (best.rot_index, ob)
        assert tuple(best.shift) == res[ob].shift
    else:
        assert scores[best.rot_index] >= order[0] - TIE
    return res, ob
