#!/usr/bin/env python3
"""Throughput of the CSNGF hot path on one MI355X.

A step is one csngf_evaluate call over a batch of rotations of the paper-scale pair
(176x176x110 float32, ~3.4 Mvoxel, FFT size 352x352x220, 1000 random rotations): every
rotation goes through resample -> NGF -> products -> forward FFT -> frequency MAC against
A's resident spectra -> inverse FFT -> exact overlap -> normalise -> argmax.  Inputs are
resident in HBM before the timed region.  Prints one JSON line.

Roofline: per-kernel device time comes from HIP events the library records around every
launch on its own stream during the timed steps; the dominant kernel's algorithmic bytes
per launch (per-rotation bytes x rotations in the launch) divided by its mean launch time
gives achieved GB/s against the 8 TB/s HBM peak.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "rotations/s at 3.4 Mvoxel (full displacement map); p50/p99 alignment latency"


def kernel_bytes(nA, nB, P, rotations_per_launch=1.0, kept=None, runs=True):
    """Algorithmic HBM bytes per rotation of each kernel family (complex64 = 8 B).

    runs: no user mask on either side, so the moving masks are runs of x per grid row found
    from the rotation (8 B per row) and the field stage writes no mask; otherwise the field
    stage writes the eroded mask (1 B per voxel) and the overlap table reads it.

    Pruned pencils: only nonzero input rows are read, H = Px/2 bins per row (the real DC and
    Nyquist bins share one complex value).  A's six conjugate spectra are read once per
    launch sequence, shared by all of its rotations, so each rotation is charged
    1/rotations_per_launch of them.  kept = (z-rows, rows) per rotation that the
    minimum-overlap pruning keeps (csngf_profile_rows): the z pass writes, the y inverse reads
    and writes, and the final pass reads only those rows (plus the overlap table once).
    Without it every displacement row is charged.
    """
    nxA, nyA, nzA = nA
    nxB, nyB, nzB = nB
    Px, Py, Pz = P
    H = Px // 2
    Wx, Wy, Wz = (nA[i] + nB[i] - 1 for i in range(3))
    kz, kr = (Wz, Wz * Wy) if kept is None else kept
    vox = nxB * nyB * nzB
    x1 = 6 * (nzB - 2) * (nyB - 2) * H * 8   # after the x pass (interior rows and slices)
    x2 = 6 * (nzB - 2) * Py * H * 8          # after the y forward pass
    spec = 6 * Pz * Py * H * 8          # A's conjugate spectra
    y3 = kz * Py * H * 8                # after the z inverse (kept z-rows)
    y4 = kr * H * 8                     # after the y inverse (kept rows)
    sat = 4 * (nxB + 1) * (nyB + 1) * (nzB + 1)
    plane = 2 if nxB * nyB < 65536 else 4   # bytes per slice prefix sum (uint16 / uint32)
    masks = 2 * 8 * nyB * nzB if runs else vox      # runs out and in, or the mask bytes in
    return {
        "fields_x": 4 * vox + x1 + (0 if runs else vox),   # B once, X1 (and the eroded mask)
        "overlap_sat": masks + 2 * plane * vox + sat,      # masks; slice prefixes out and back; table out
        "y_forward": x1 + x2,
        "z_mac_inverse": x2 + spec / rotations_per_launch + y3,
        "y_inverse": y3 + y4,
        "x_c2r_argmax": y4 + (sat if kept is not None else 0),
    }


# FP32 vector peak without packed FP32 (which this code does not use): 256 CUs x 4 SIMDs x 16
# lanes x 2 flop (fma) x 2.4 GHz
VALU_FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def plan_radices(L):
    """The FFT engine's factorisation of L: odd radices first (11, 7, 5, 3), then 8, 4, 2."""
    n, rs = L, []
    for q in (11, 7, 5, 3, 8, 4, 2):
        while n % q == 0:
            rs.append(q)
            n //= q
    return rs


def dft_flops(R, pruned):
    """Real flops of one radix-R butterfly as the engine computes it (fma = 2); pruned: the
    upper half of the inputs is zero (first stage of a zero-padded transform)."""
    if R == 2:
        return 0 if pruned else 4
    if R == 4:
        return 8 if pruned else 16
    if R == 8:
        return 40 if pruned else 56
    h = (R - 1) // 2    # odd R: pairs x_m with x_(R-m)
    return (6 if pruned else 10) * h + 8 * h * h


def transform_flops(L, pruned_first):
    """Flops of one length-L complex transform: butterflies plus twiddle products (6 flops
    each) at every stage after the first."""
    f, ns = 0, 1
    for s, R in enumerate(plan_radices(L)):
        f += (L // R) * (dft_flops(R, pruned_first and s == 0) + (6 * (R - 1) if ns > 1 else 0))
        ns *= R
    return f


def zpass_flops(nB, P, nf=6):
    """Algorithmic flops per rotation of the z pass: for every (ky, kx) pencil, nf pruned
    forward transforms, nf complex multiply-accumulates per bin, one full inverse."""
    Px, Py, Pz = P
    pruned = 2 * (nB[2] - 2) <= Pz
    return Py * (Px // 2) * (nf * (transform_flops(Pz, pruned) + 8 * Pz) + transform_flops(Pz, False))


def paper_yardstick(nA, nB, P):
    """The fixed per-rotation byte model of the method as the paper states it (Sec. 3.1: 7
    forward and 2 inverse zero-padded real 3-D FFTs per rotation with A's 7 spectra cached and
    read once per rotation), as three pruned complex64 pencil passes each: x writes and y
    reads nz ny (Px/2+1) bins per field, y writes and z reads nz Py (Px/2+1), each inverse
    moves Pz Py (Px/2+1) four times; plus B once.  A design that moves fewer bytes (here: no
    mask transforms, spectra shared per launch, pruned inverse rows) shows up as a fraction
    of this yardstick above its HBM-bound rate."""
    nxB, nyB, nzB = nB
    Px, Py, Pz = P
    H1 = Px // 2 + 1
    f = 7
    x_out = f * nzB * nyB * H1 * 8
    y_out = f * nzB * Py * H1 * 8
    spec = f * Pz * Py * H1 * 8
    inv = 2 * 4 * Pz * Py * H1 * 8
    return 2 * x_out + 2 * y_out + spec + inv + 4 * nxB * nyB * nzB


# Sec. 5.2, Table 3: FFT-based CSNGF, one evaluation, seconds, by cube side (RTX 3090; context)
PAPER_TABLE3_S = {8: 0.002, 16: 0.002, 32: 0.002, 64: 0.008, 128: 0.088}


KERNEL_SOURCE = {"z_mac_inverse": "k_zpass", "y_forward": "k_pencil", "y_inverse": "k_pencil",
                 "fields_x": "k_fields_x", "x_c2r_argmax": "k_final_x"}


def source_hash(kernel="z_mac_inverse"):
    """Hash of the FFT engine plus the source text of the kernel's own function."""
    csrc = os.path.join(ROOT, "paper_2110_10156_amd", "csrc")
    h = hashlib.sha256(open(os.path.join(csrc, "csngf_fft.hpp"), "rb").read())
    text = open(os.path.join(csrc, "csngf_kernels.hpp")).read()
    name = KERNEL_SOURCE.get(kernel, kernel)
    m = re.search(r"void " + re.escape(name) + r"\(.*?\n}\n", text, flags=re.S)
    h.update((m.group(0) if m else text).encode())
    return h.hexdigest()[:16]


def read_traffic(kernel, workload):
    """Measured HBM bytes per launch from a committed rocprofv3 PMC summary, if it was taken
    on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_hash:\s*([0-9a-f]+)", text)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    r = re.search(r"rotations_per_launch:\s*([0-9]+)", text)
    if not (m and b and r) or m.group(1) != source_hash(kernel):
        return None
    return float(b.group(1)), int(r.group(1))


def cpu_baseline(pair, n_rot):
    """The FP64 oracle timed per rotation on the host: A's fixed fields once (untimed, as the
    GPU context holds them), then for each rotation the oracle's own steps in its order
    (resample + NGF, Eq. (6)-(8) FFT correlation, normalise, argmax).  Median over n_rot
    rotations with the FFTs on all permitted threads, and again on one thread."""
    from oracle import csngf_oracle as O
    rots = pair.rotations[:n_rot]
    fa = O.fixed_fields(pair.A)
    count_a = int(np.count_nonzero(fa.mask))

    def one(R):
        fb = O.moving_fields(pair.B, O.quantize_rotation(R))
        S, N = O.correlation_maps_fft(fa, fb, pair.pad)
        C, _ = O.normalise(S, N, count_a, int(np.count_nonzero(fb.mask)))
        O.argmax_map(C)

    def median_time(workers):
        saved = O.WORKERS
        O.WORKERS = workers
        try:
            ts = []
            for R in rots:
                t0 = time.perf_counter()
                one(R)
                ts.append(time.perf_counter() - t0)
        finally:
            O.WORKERS = saved
        return float(np.median(ts))

    t_all = median_time(O.WORKERS)
    t_one = median_time(1)
    return {"value": round(1.0 / t_all, 4), "unit": "rotations/s", "cores": int(O.WORKERS), "kind": "oracle",
            "sample": f"median of {n_rot} rotations of the 176x176x110 pair at FFT size 352x352x220 "
                      f"(FP64 numpy/scipy; {t_all:.2f} s per rotation with FFTs on {O.WORKERS} threads, "
                      f"the rest single-threaded)",
            "one_thread": {"value": round(1.0 / t_one, 4), "unit": "rotations/s", "cores": 1,
                           "seconds_per_rotation": round(t_one, 3)}}


def secondary_lines(torch, bd, synth, n_small=2048, n_mid=512, sweep_reps=20):
    """Throughput of the 32^3 pair (FFT 64^3) and the 96x96x64 pair (FFT 192x192x128), plain
    (one rotation per launch sequence) and batched (automatic slots), and the per-evaluation
    time by cube side (Sec. 5.2, Table 3 sweep: sides 8..128, FFT 2n per axis)."""
    dev = torch.device("cuda:0")
    out = {}

    def rate(ctx, B, rots):
        ctx.evaluate(B, rots[:8])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.evaluate(B, rots)
        return len(rots) / (time.perf_counter() - t0)

    for name, pair, n in (("32x32x32", synth.config0(), n_small), ("96x96x64", synth.config1(n_random=0), n_mid)):
        A = torch.from_numpy(pair.A).to(dev)
        B = torch.from_numpy(pair.B).to(dev)
        rots = synth.random_rotations(n, 4242)
        with bd.Context(A, pair.dims_b, pad=pair.pad, batch=1) as c1, bd.Context(A, pair.dims_b, pad=pair.pad) as cb:
            plain = rate(c1, B, rots[: max(64, n // 8)])
            batched = rate(cb, B, rots)
            out[name] = {"fft_size": list(cb.info().pad), "slots": cb.info().batch,
                         "plain_rotations_per_s": round(plain, 1), "batched_rotations_per_s": round(batched, 1)}
        print(f"[bench] {name}: plain {plain:.1f} rot/s, batched {batched:.1f} rot/s", file=sys.stderr, flush=True)
    sweep = {}
    for side in sorted(PAPER_TABLE3_S):
        pair = synth.cube_pair(side)
        A = torch.from_numpy(pair.A).to(dev)
        B = torch.from_numpy(pair.B).to(dev)
        R1 = np.eye(3)[None]
        with bd.Context(A, pair.dims_b, pad=pair.pad, batch=1) as c1, bd.Context(A, pair.dims_b, pad=pair.pad) as cb:
            c1.evaluate(B, R1)
            ts = []
            for _ in range(sweep_reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                c1.evaluate(B, R1)        # one evaluation, host to host
                ts.append(time.perf_counter() - t0)
            batched = rate(cb, B, synth.random_rotations(256, 4243))
        sweep[str(side)] = {"fft_size": list(pair.pad), "ms_per_evaluation": round(float(np.median(ts)) * 1e3, 3),
                            "batched_ms_per_rotation": round(1e3 / batched, 4),
                            "paper_table3_ms_rtx3090": PAPER_TABLE3_S[side] * 1e3}
        print(f"[bench] cube {side}: {sweep[str(side)]}", file=sys.stderr, flush=True)
    out["cube_side_sweep"] = sweep
    return out


def many_pairs(torch, bd, synth, big_pair, n_pairs, n_rot, budget_gib=160.0):
    """Uneven-size batch: n_pairs pairs with sizes drawn uniformly from synth.MIXED_SHAPES
    (seed 3000 + i), n_rot random rotations each.  One phantom pair per distinct size stands
    in for every pair of that size (throughput depends on sizes only).
    Sequential: pair after pair, one synchronous evaluation each, default parameters (the
    evaluation calls are timed, context creation is not).
    Concurrent: all contexts alive, each on its own stream, every evaluation in flight at
    once, graph replay, autotuned (P, slots, launch shapes); if the contexts' workspaces
    together exceed budget_gib of HBM, every context's slots are scaled down alike.
    Sequential, tuned: the concurrent mode's contexts, one pair after another.
    Per size: the sequential rate and the autotuned rate of one pair alone (graphs)."""
    dev = torch.device("cuda:0")
    sizes = [synth.MIXED_SHAPES[int(np.random.default_rng(3000 + i).integers(0, len(synth.MIXED_SHAPES)))]
             for i in range(n_pairs)]
    vols = {}
    for sz in sorted(set(sizes)):
        p = big_pair if sz == big_pair.dims_a else synth.mixed_pair_of_size(sz)
        vols[sz] = (torch.from_numpy(p.A).to(dev), torch.from_numpy(p.B).to(dev))
    rots = [synth.random_rotations(n_rot, 5000 + i) for i in range(n_pairs)]
    tuned, tuned_rate, mem = {}, {}, {}
    for sz in sorted(set(sizes)):
        A, B = vols[sz]
        cfg, rate = bd.autotune(A, B, n_probe=64, graphs=True)
        with bd.Context(A, bd.dims_of(B), pad=cfg["pad"], batch=1) as c1:
            mem[sz] = (c1.info().spectra_bytes, c1.info().workspace_bytes)
        tuned[sz], tuned_rate[sz] = cfg, rate
    need = sum(mem[sz][0] + tuned[sz]["batch"] * mem[sz][1] for sz in sizes)
    scale = min(1.0, budget_gib * 2**30 / need)
    for sz in tuned:
        tuned[sz]["batch"] = int(max(1, tuned[sz]["batch"] * scale))
    torch.cuda.synchronize()
    key = lambda s: f"{s[0]}x{s[1]}x{s[2]}"
    out = {"pairs": n_pairs, "rotations_per_pair": n_rot,
           "sizes": {key(s): sizes.count(s) for s in sorted(set(sizes))},
           "concurrent_params": {key(s): tuned[s] for s in sorted(set(sizes))},
           "slot_scale": round(scale, 3)}
    # sequential
    total, per_size = 0.0, {}
    for sz, r in zip(sizes, rots):
        A, B = vols[sz]
        with bd.Context(A, bd.dims_of(B)) as c:
            c.evaluate(B, r[:8])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.evaluate(B, r)
            dt = time.perf_counter() - t0
            total += dt
            per_size.setdefault(sz, []).append(dt)
    out["sequential_rotations_per_s"] = round(n_pairs * n_rot / total, 1)
    print(f"[bench] many pairs sequential: {n_pairs * n_rot / total:.1f} rot/s", file=sys.stderr, flush=True)
    # one pair of each size alone with its tuned configuration (graphs, unscaled slots)
    alone = {}
    for sz in sorted(set(sizes)):
        A, B = vols[sz]
        cfg = dict(tuned[sz])
        cfg["batch"] = int(round(cfg["batch"] / scale)) if scale < 1.0 else cfg["batch"]
        with bd.Context(A, bd.dims_of(B), graphs=True, **cfg) as c:
            r = rots[sizes.index(sz)]
            c.evaluate(B, r[:c.info().batch])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.evaluate(B, r)
            alone[sz] = n_rot / (time.perf_counter() - t0)
    out["per_size"] = {key(s): {"sequential_rotations_per_s": round(len(per_size[s]) * n_rot / sum(per_size[s]), 1),
                                "tuned_alone_rotations_per_s": round(alone[s], 1),
                                "autotune_probe_rotations_per_s": round(tuned_rate[s], 1)}
                       for s in sorted(set(sizes))}
    # concurrent
    ctxs = [bd.Context(vols[sz][0], bd.dims_of(vols[sz][1]), graphs=True, **tuned[sz]) for sz in sizes]
    for c, sz, r in zip(ctxs, sizes, rots):            # warm-up: graph recording, first launches
        c.evaluate(vols[sz][1], r[:c.info().batch])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, sz, r in zip(ctxs, sizes, rots):
        c.evaluate_async(vols[sz][1], r)
    for c in ctxs:
        c.wait()
    dt = time.perf_counter() - t0
    out["concurrent_rotations_per_s"] = round(n_pairs * n_rot / dt, 1)
    print(f"[bench] many pairs concurrent: {n_pairs * n_rot / dt:.1f} rot/s", file=sys.stderr, flush=True)
    # the same contexts (tuned, graphs) one pair after another
    t0 = time.perf_counter()
    for c, sz, r in zip(ctxs, sizes, rots):
        c.evaluate(vols[sz][1], r)
    dt = time.perf_counter() - t0
    for c in ctxs:
        c.close()
    out["sequential_tuned_rotations_per_s"] = round(n_pairs * n_rot / dt, 1)
    print(f"[bench] many pairs sequential, tuned + graphs: {n_pairs * n_rot / dt:.1f} rot/s", file=sys.stderr,
          flush=True)
    return out


def requests_for_rate(rate, cap):
    """Requests per rate: about 8 s of arrivals, at least 12 and at most cap."""
    return int(max(12, min(cap, round(8 * rate))))


def serving(torch, bd, synth, big_pair, rates, n_cap, n_rot, miss_rate=0.5, budget_gib=96.0):
    """Poisson request streams.  Each request pairs a fixed volume of a size drawn uniformly
    from synth.MIXED_SHAPES with its moving volume and n_rot random rotations.  With
    probability miss_rate the request brings a fixed volume the server has never seen (the
    size's phantom plus fresh noise, so its spectra must be computed and a context admitted),
    otherwise it reuses the size's phantom, whose context is cached.  Latency is finish -
    arrival on the server clock, reported for all requests and separately for cache hits and
    misses.  Volumes are built on the device before each stream starts."""
    from paper_2110_10156_amd import serve
    dev = torch.device("cuda:0")
    vols = {}
    for sz in synth.MIXED_SHAPES:
        p = big_pair if sz == big_pair.dims_a else synth.mixed_pair_of_size(sz)
        vols[sz] = (torch.from_numpy(p.A).to(dev), torch.from_numpy(p.B).to(dev))
    out = {"rotations_per_request": n_rot, "hbm_budget_gib": budget_gib, "miss_rate": miss_rate,
           "what": "latency = finish - arrival; a miss computes a new fixed volume's spectra"}
    srv = serve.Server(hbm_budget=int(budget_gib * 2**30))
    warm = [serve.Request(-1 - i, str(sz), *vols[sz], synth.random_rotations(8, 77)) for i, sz in
            enumerate(synth.MIXED_SHAPES)]
    serve.run_stream(srv, lambda i: warm[i], np.zeros(len(warm)))
    for rate in rates:
        n_req = requests_for_rate(rate, n_cap)
        rng = np.random.default_rng(int(rate * 100))
        sizes = [synth.MIXED_SHAPES[int(rng.integers(0, len(synth.MIXED_SHAPES)))] for _ in range(n_req)]
        miss = rng.random(n_req) < miss_rate
        gen = torch.Generator(device=dev)
        gen.manual_seed(int(rate * 1000))
        fixed = []
        for i, sz in enumerate(sizes):
            A0 = vols[sz][0]
            if miss[i]:
                A1 = A0 + 1e-3 * torch.randn(A0.shape, device=dev, generator=gen)
                fixed.append((f"{sz}-{rate:g}-{i}", A1))
            else:
                fixed.append((str(sz), A0))
        torch.cuda.synchronize()
        rots = [synth.random_rotations(n_rot, 7000 + i) for i in range(n_req)]
        arr = serve.poisson_arrivals(rate, n_req, seed=int(rate * 10))
        res = serve.run_stream(srv, lambda i: serve.Request(i, fixed[i][0], fixed[i][1], vols[sizes[i]][1],
                                                            rots[i]), arr)
        summ = serve.summarize(res, n_rot)
        out[f"{rate:g}_req_per_s"] = summ
        print(f"[bench] serving {rate:g} req/s: {summ}", file=sys.stderr, flush=True)
        del fixed
    out["contexts_created"] = srv.stats.created
    out["contexts_evicted"] = srv.stats.evicted
    out["peak_in_flight"] = srv.stats.peak_inflight
    srv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rotations", type=int, default=1000, help="rotations per step")
    ap.add_argument("--batch", type=int, default=0, help="rotation slots in flight (0 = library default)")
    ap.add_argument("--cpu-rotations", type=int, default=3,
                    help="oracle sample: rotations timed (median), on all threads and on one (0 = skip)")
    ap.add_argument("--plain-rotations", type=int, default=64,
                    help="rotations timed on the one-rotation-per-launch path (0 = skip)")
    ap.add_argument("--fp64-rotations", type=int, default=96,
                    help="rotations timed with the FP64 correlation (CSNGF_FP64); 0 skips")
    ap.add_argument("--usngf-rotations", type=int, default=200,
                    help="rotations timed with the unsquared measure, Eq. (3) (0 = skip)")
    ap.add_argument("--align-runs", type=int, default=5,
                    help="full global alignments (paper schedule) timed for p50/p99 latency (0 = skip)")
    ap.add_argument("--batched-pairs", type=int, default=32,
                    help="uneven volume pairs (48^3 .. 176x176x110) for the many-pairs measurement (0 = skip)")
    ap.add_argument("--batched-rotations", type=int, default=256, help="rotations per pair in that measurement")
    ap.add_argument("--serve-rates", default="1,2,5,10,20",
                    help="Poisson arrival rates (requests/s) for the serving measurement ('' = skip)")
    ap.add_argument("--serve-requests", type=int, default=100,
                    help="most requests per rate (each rate gets about 8 s of arrivals, at least 12)")
    ap.add_argument("--serve-miss-rate", type=float, default=0.5,
                    help="fraction of requests that bring a fixed volume the server has not seen")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 32^3 / 96x96x64 throughput lines and the cube-side sweep")
    ap.add_argument("--serve-rotations", type=int, default=200, help="rotations per request")
    ap.add_argument("--no-profile", action="store_true", help="do not record per-kernel events")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2110_10156_amd import binding as bd
    from paper_2110_10156_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    pair = synth.config2(n_random=args.rotations)
    rots = pair.rotations[:args.rotations]
    A = torch.from_numpy(pair.A).to(dev)
    B = torch.from_numpy(pair.B).to(dev)
    torch.cuda.synchronize()

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * 2**20 // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print(f"[bench] calibration copy of {args.calib_copy_mib} MiB done", file=sys.stderr, flush=True)

    ctx = bd.Context(A, pair.dims_b, pad=pair.pad, batch=args.batch)
    info = ctx.info()
    slots = info.batch
    print(f"[bench] ctx ready: P={tuple(info.pad)} slots={slots} "
          f"spectra {info.spectra_bytes / 2**20:.0f} MiB workspace {info.workspace_bytes / 2**30:.2f} GiB",
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        ctx.evaluate(B, rots)
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    if not args.no_profile:
        ctx.profile_reset()
        ctx.profile_enable(True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        per, best = ctx.evaluate(B, rots)     # synchronous: returns with results on the host
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"[bench] timed {args.steps} steps", file=sys.stderr, flush=True)
    stats = {}
    if not args.no_profile:
        stats = ctx.profile_read()
        ctx.profile_enable(False)
    elapsed = t1 - t0
    value = args.steps * len(rots) / elapsed

    roofline = roofline_fields = roofline_valu = None
    kept = None
    seq_rot = len(rots) / math.ceil(len(rots) / slots)   # mean rotations per launch sequence
    if stats:
        kz, kr, nr = ctx.profile_rows()
        if nr > 0:
            kept = (kz / nr, kr / nr)
    kb = kernel_bytes(pair.dims_a, pair.dims_b, tuple(info.pad), seq_rot, kept)

    def roof(kernel):
        launches, ms = stats[kernel]
        per_launch_rot = len(rots) * args.steps / launches
        alg = kb[kernel] * per_launch_rot
        avg_s = ms / launches / 1e3
        achieved = alg / avg_s / 1e9
        tr = read_traffic(kernel, "176x176x110")
        traffic = None if tr is None else tr[0] / tr[1] * per_launch_rot
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
                "avg_launch_ms": round(avg_s * 1e3, 4), "rotations_per_launch": per_launch_rot,
                "alg_bytes_per_launch": alg}

    if stats:
        dom = max((k for k in kb if stats.get(k, (0, 0))[0] > 0), key=lambda k: stats[k][1])
        roofline = roof(dom)
        roofline["kernels_ms_per_rotation"] = {k: round(v[1] / (len(rots) * args.steps), 5)
                                               for k, v in stats.items() if v[0]}
        if kept is not None:
            roofline["kept_rows_per_rotation"] = {"z_rows": round(kept[0], 2), "rows": round(kept[1], 1),
                                                  "of_z_rows": pair.dims_a[2] + pair.dims_b[2] - 1,
                                                  "of_rows": (pair.dims_a[2] + pair.dims_b[2] - 1)
                                                  * (pair.dims_a[1] + pair.dims_b[1] - 1)}
        if stats.get("fields_x", (0, 0))[0] > 0:
            roofline_fields = roof("fields_x")
        if stats.get("z_mac_inverse", (0, 0))[0] > 0:
            # the z pass is bound by vector-ALU issue (counter summary): its arithmetic against
            # the FP32 vector peak without packed math
            launches, ms = stats["z_mac_inverse"]
            per_launch_rot = len(rots) * args.steps / launches
            fl = zpass_flops(pair.dims_b, tuple(info.pad)) * per_launch_rot
            tf = fl / (ms / launches / 1e3) / 1e12
            roofline_valu = {"bound": "alu", "achieved": round(tf, 2), "peak": round(VALU_FP32_PEAK_TFLOPS, 2),
                             "unit": "TFLOP/s", "frac": round(tf / VALU_FP32_PEAK_TFLOPS, 4),
                             "kernel": "z_mac_inverse", "alg_flops_per_launch": fl,
                             "peak_what": "FP32 vector fma, packed FP32 not used: 256 CUs x 4 SIMDs x 16 lanes x "
                                          "2 flop x 2.4 GHz"}
        print(f"[bench] kernel ms/rotation: {roofline['kernels_ms_per_rotation']}", file=sys.stderr, flush=True)

    plain = None
    if args.plain_rotations > 0:
        with bd.Context(A, pair.dims_b, pad=pair.pad, batch=1) as pctx:
            pr = rots[:args.plain_rotations]
            pctx.evaluate(B, pr[:4])
            torch.cuda.synchronize()
            ts = time.perf_counter()
            pctx.evaluate(B, pr)
            torch.cuda.synchronize()
            plain = len(pr) / (time.perf_counter() - ts)
        print(f"[bench] plain path {plain:.1f} rot/s", file=sys.stderr, flush=True)

    usngf = None
    if args.usngf_rotations > 0:
        with bd.Context(A, pair.dims_b, pad=pair.pad, batch=args.batch, measure="unsquared") as uctx:
            ur = rots[:args.usngf_rotations]
            uctx.evaluate(B, ur[:16])
            torch.cuda.synchronize()
            ts = time.perf_counter()
            uctx.evaluate(B, ur)
            torch.cuda.synchronize()
            usngf = len(ur) / (time.perf_counter() - ts)
        print(f"[bench] unsquared measure {usngf:.1f} rot/s", file=sys.stderr, flush=True)

    fp64 = None
    if args.fp64_rotations > 0:
        # the same workload with the transforms in FP64 (CSNGF_FP64): the exact-at-small-overlap mode
        with bd.Context(A, pair.dims_b, pad=pair.pad, batch=args.batch, fp64=True) as dctx:
            dr = rots[:args.fp64_rotations]
            dctx.evaluate(B, dr[:8])
            torch.cuda.synchronize()
            ts = time.perf_counter()
            dctx.evaluate(B, dr)
            torch.cuda.synchronize()
            fp64 = len(dr) / (time.perf_counter() - ts)
            fp64_slots = dctx.info().batch
        print(f"[bench] FP64 correlation {fp64:.1f} rot/s ({fp64_slots} slots)", file=sys.stderr, flush=True)

    align_stats = None
    if args.align_runs > 0:
        from paper_2110_10156_amd import align as al

        def runs(ev):
            alat, dEs, ok = [], [], 0
            for r in range(args.align_runs):
                torch.cuda.synchronize()
                res = al.align(A, B, al.PAPER_SCHEDULE, seed=r, evaluator=ev)
                alat.append(res.seconds)
                dE = al.corner_distance(pair.A.shape, pair.B.shape, pair.true_rotation, pair.true_shift, res.R,
                                        res.shift)
                dEs.append(dE)
                ok += dE < 5.0
                print(f"[bench] alignment {r}: {res.seconds:.3f} s, d_E {dE:.2f} vx", file=sys.stderr, flush=True)
            return np.array(alat) * 1e3, dEs, ok

        # tuned: one autotune per pair of level shapes, in the warm-up alignment (cached after)
        ev = al.GpuEvaluator(tune=True)
        al.align(A, B, al.PAPER_SCHEDULE, seed=1000, evaluator=ev)   # warm-up: kernels, tuning
        la, dEs, ok = runs(ev)
        plain_ev = al.GpuEvaluator()
        al.align(A, B, al.PAPER_SCHEDULE, seed=1000, evaluator=plain_ev)
        lu, _, _ = runs(plain_ev)
        align_stats = {"p50_ms": round(float(np.percentile(la, 50)), 1), "p99_ms": round(float(np.percentile(la, 99)), 1),
                       "runs": args.align_runs, "success_dE_lt_5": ok, "median_dE_vx": round(float(np.median(dEs)), 2),
                       "evaluations": sum(p + a for p, a in zip(al.PAPER_SCHEDULE["p"], al.PAPER_SCHEDULE["a"])),
                       "untuned_p50_ms": round(float(np.percentile(lu, 50)), 1),
                       "untuned_p99_ms": round(float(np.percentile(lu, 99)), 1),
                       "tuned_configs": {f"{k[0]}/{k[1]}": v for k, v in ev.tuned.items()},
                       "what": "global rigid alignment of the 176x176x110 pair with the paper's pyramid schedule "
                               "(host to host, seeds 0..runs-1); tuned: FFT size and launch shapes per level shape "
                               "from the autotuner, run once per shape in a warm-up alignment; untuned: the "
                               "automatic choices"}

    batched = None
    if args.batched_pairs > 0:
        batched = many_pairs(torch, bd, synth, pair, args.batched_pairs, args.batched_rotations)

    served = None
    if args.serve_rates:
        served = serving(torch, bd, synth, pair, [float(r) for r in args.serve_rates.split(",")],
                         args.serve_requests, args.serve_rotations, miss_rate=args.serve_miss_rate)

    secondary = None
    if not args.no_secondary:
        secondary = secondary_lines(torch, bd, synth)

    cpu = None
    if args.cpu_rotations > 0:
        cpu = cpu_baseline(pair, args.cpu_rotations)
        print(f"[bench] oracle {cpu['value']:.3f} rot/s", file=sys.stderr, flush=True)

    lat_ms = np.array(lat) * 1e3
    yard = sum(kb.values())
    paper_yard = paper_yardstick(pair.dims_a, pair.dims_b, tuple(info.pad))
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "rotations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "176x176x110 float32 pair (3.4 Mvoxel), 4-class shell phantom, "
                               f"{len(rots)} random rotations per step, FFT 352x352x220, full displacement map",
                   "rotations_per_step": len(rots), "fft_size": list(info.pad), "slots": slots},
        "alignment_latency": align_stats,
        "many_pairs": batched,
        "serving": served,
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                       "p99": round(float(np.percentile(lat_ms, 99)), 3),
                       "what": f"one csngf_evaluate call of {len(rots)} rotations, host to host"},
        "plain_rotations_per_s": None if plain is None else round(plain, 2),
        "usngf_rotations_per_s": None if usngf is None else round(usngf, 2),
        "fp64_rotations_per_s": None if fp64 is None else round(fp64, 2),
        "path_bytes_per_rotation": yard,
        "path_bytes_kept_rows": kept is not None,
        "path_hbm_frac": round(yard * value / (HBM_PEAK_GBS * 1e9), 4),
        "yardstick_bytes_per_rotation": paper_yard,
        "yardstick_frac": round(paper_yard * value / (HBM_PEAK_GBS * 1e9), 4),
        "yardstick_what": "fixed byte model of the paper's 7 forward + 2 inverse FFTs with A's 7 spectra read per "
                          "rotation; this design skips the mask transforms, shares A's spectra per launch and "
                          "prunes inverse rows, so this fraction can exceed what its own kernels move",
        "secondary": secondary,
        "best": {"rot_index": best.rot_index, "shift": list(best.shift), "score": best.score},
        "roofline": roofline,
        "roofline_field_stage": roofline_fields,
        "roofline_z_pass_valu": roofline_valu,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
