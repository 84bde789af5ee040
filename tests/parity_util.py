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


# ------------------------------------------------------------------ many rotations in parallel
# The oracle's per-rotation steps (resample + NGF of B, Eq. (6)-(8) correlation, normalise,
# argmax) for many rotations, spread over worker processes (spawned: they load numpy and the
# oracle only).  Each worker holds A's fields once; per rotation it returns what the bar needs,
# including C and N at the displacement the GPU picked.
_W = {}


def _worker_init(A, B, mask_a, mask_b, gamma, measure, P, fft_threads):
    O.WORKERS = fft_threads
    fa = O.fixed_fields(A, mask_a)
    _W.update(A=A, B=B, mask_b=mask_b, gamma=gamma, measure=measure, P=P, fa=fa,
              count_a=int(np.count_nonzero(fa.mask)))


def _worker_rotation(R, gpu_shift):
    fa = _W["fa"]
    fb = O.moving_fields(_W["B"], O.quantize_rotation(R), _W["mask_b"])
    S, N = O.correlation_maps_fft(fa, fb, _W["P"], _W["measure"])
    C, _ = O.normalise(S, N, _W["count_a"], int(np.count_nonzero(fb.mask)), _W["gamma"])
    am = O.argmax_map(C)
    nza, nya, nxa = fa.mask.shape
    if am is None:
        return dict(valid=False)
    score, flat = am
    iz, iy, ix = np.unravel_index(flat, C.shape)
    v = np.isfinite(C)
    top = np.partition(C[v], -2)[-2:] if v.sum() > 1 else None
    gz, gy, gx = gpu_shift[2] + nza - 1, gpu_shift[1] + nya - 1, gpu_shift[0] + nxa - 1
    inside = 0 <= gz < C.shape[0] and 0 <= gy < C.shape[1] and 0 <= gx < C.shape[2]
    return dict(valid=True, score=float(score),
                shift=(int(ix) - (nxa - 1), int(iy) - (nya - 1), int(iz) - (nza - 1)),
                overlap=int(N[iz, iy, ix]), gap=None if top is None else float(top[1] - top[0]),
                c_at_gpu=float(C[gz, gy, gx]) if inside else -np.inf,
                n_at_gpu=int(N[gz, gy, gx]) if inside else -1)


def check_against_oracle_parallel(A, B, rotations, per, best, P=None, gamma=0.5, measure="squared", mask_b=None,
                                  mask_a=None, procs=4):
    """check_against_oracle's bar for every rotation, the oracle run in `procs` processes."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cores = os.cpu_count() or 1
    cores = min(cores, 16)
    procs = max(1, min(procs, cores))
    rots = np.asarray(rotations, dtype=np.float64).reshape(-1, 3, 3)
    args = (np.asarray(A), np.asarray(B), mask_a, mask_b, gamma, measure, P, max(1, cores // procs))
    with cf.ProcessPoolExecutor(max_workers=procs, mp_context=mp.get_context("spawn"),
                                initializer=_worker_init, initargs=args) as ex:
        res = list(ex.map(_worker_rotation, list(rots), [tuple(g.shift) for g in per]))
    scores = []
    for i, (g, r) in enumerate(zip(per, res)):
        assert bool(g.valid) == r["valid"], (i, g.valid, r["valid"])
        if not r["valid"]:
            scores.append(-np.inf)
            continue
        scores.append(r["score"])
        assert abs(float(g.score) - r["score"]) <= CTOL, (i, float(g.score), r["score"])
        if r["gap"] is None or r["gap"] >= TIE:
            assert tuple(g.shift) == r["shift"], (i, tuple(g.shift), r["shift"])
        else:
            assert r["c_at_gpu"] >= r["score"] - TIE, (i, tuple(g.shift), r["shift"])
        assert g.overlap == r["n_at_gpu"], (i, g.overlap, r["n_at_gpu"])
    scores = np.array(scores)
    fin = scores[np.isfinite(scores)]
    if fin.size == 0:
        assert best.rot_index == -1
        return res
    ob = int(np.argmax(scores))   # first index among equal scores: the smaller rotation index
    order = np.sort(fin)[::-1]
    if order.size < 2 or order[0] - order[1] >= TIE:
        assert best.rot_index == ob, (best.rot_index, ob)
        assert tuple(best.shift) == res[ob]["shift"]
    else:
        assert scores[best.rot_index] >= order[0] - TIE
    return res
