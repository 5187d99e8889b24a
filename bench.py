"""Throughput of the Voronoi point-inclusion path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--points M]

Workload (one "step"): the streaming sweep -- six convex polygons with 3, 4,
8, 16, 32 and 64 vertices on a circle of radius 1, each tested against its
own 2^28 float32 points uniform in [-1.5, 1.5]^2 of which 1% lie within 1e-6
of an edge.  Each polygon is one call of the C ABI's pip_voronoi (binary64
generator derivation, float32 screen of every edge's margin with a proven
band, binary64 recheck, packed labels), all on one stream with the inputs
resident in HBM.  Every point meets every edge, as in the paper's own
comparison of the tests (Section 6.2); the radial pre-screen, a culling
layer in front of the test, is timed and reported apart.

Prints one JSON line: whole-step throughput in G point-polygon tests/s, the
roofline of the dominant kernel (measured with HIP events on the launch
stream), per-polygon figures (with the float32 margin error against the
binary64 one and the share of points the band sends to binary64), sign of
offset, ray crossing and the float32-only kernel for comparison, label
mismatches of all three tests against the FP64 oracle over the whole sweep,
and the oracle's own throughput on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (dense)
BYTES_PER_TEST = 8.125         # float2 point in + 1 label bit out
NS = (3, 4, 8, 16, 32, 64)


# device code of the single-polygon streaming kernels (whose HBM traffic
# profiles/hbm_traffic.json records); the shared declarations header is left out
STREAM_SOURCES = ("device.hpp", "radial.hpp", "stream.hip", "stream32.hpp", "stream_mfma.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2007_15385_amd", "csrc")
    for fn in STREAM_SOURCES:
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(fn.encode() + f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel_key: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash():
        return None
    e = d.get("kernels", {}).get(kernel_key)
    return None if e is None else float(e["bytes_per_launch"])


def _counter_rows(d: str, counter: str):
    """(dispatch id, kernel name, value summed over the counter's rows) per
    dispatch of a rocprofv3 --pmc csv run, in dispatch order."""
    import csv
    import glob
    f = glob.glob(os.path.join(d, "*counter_collection.csv"))[0]
    agg = {}
    with open(f) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            did = int(r["Dispatch_Id"])
            agg.setdefault(did, [r["Kernel_Name"], 0.0])[1] += float(r["Counter_Value"])
    return [(k, agg[k][0], agg[k][1]) for k in sorted(agg)]


def ingest_counters(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir) -> int:
    """profiles/hbm_traffic.json from counter runs of `--traffic-run` (one
    Voronoi launch per n, in NS order) and `--copy-probe` (1 GiB copies),
    each counter scaled by what it reads for the copy of known size."""
    copy_bytes = float(1 << 30)
    cf = max(v for _, name, v in _counter_rows(copy_fetch_dir, "FETCH_SIZE"))
    cw = max(v for _, name, v in _counter_rows(copy_write_dir, "WRITE_SIZE"))
    sf, sw = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)

    def voronoi(rows):
        return [v for _, name, v in rows
                if "k_stream32<0>" in name or "k_stream_mfma<0," in name or "k_stream32_radial" in name]
    fe = voronoi(_counter_rows(fetch_dir, "FETCH_SIZE"))
    wr = voronoi(_counter_rows(write_dir, "WRITE_SIZE"))
    if len(fe) != len(NS) or len(wr) != len(NS):
        print(f"expected {len(NS)} Voronoi dispatches, got {len(fe)} / {len(wr)}", file=sys.stderr)
        return 1
    m = 1 << 28
    out = {"source_hash": kernel_source_hash(),
           "scale": {"FETCH_SIZE": round(sf, 4), "WRITE_SIZE": round(sw, 4)},
           "algorithmic_bytes_per_launch": BYTES_PER_TEST * m, "kernels": {}}
    print("| n | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (scaled) | / algorithmic |")
    print("|---|---|---|---|---|")
    for n, f, w in zip(NS, fe, wr):
        b = f * 1024.0 * sf + w * 1024.0 * sw
        out["kernels"][f"voronoi_f32_n{n}"] = {"fetch_kib": f, "write_kib": w,
                                               "bytes_per_launch": round(b)}
        print(f"| {n} | {f:.0f} | {w:.0f} | {b:.4g} | {b / (BYTES_PER_TEST * m):.3f} |")
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"scale FETCH_SIZE {sf:.4f}, WRITE_SIZE {sw:.4f}; wrote profiles/hbm_traffic.json")
    return 0


def annulus_fraction(P, torch, V, Q, sample=1 << 20):
    """Share of the first `sample` points that the radial pre-screen leaves to
    the per-edge screen (float64 evaluation of its tests on the host; a
    diagnostic, not a label)."""
    b = P.pip_voronoi_radial_bounds(torch.from_numpy(V).cuda()).cpu().numpy()
    p0 = P.polygon_to_generators(torch.from_numpy(V).cuda()).cpu().numpy()[0]
    q = Q[:sample]
    X = (q[:, 0] - np.float32(p0[0])).astype(np.float32)
    Y = (q[:, 1] - np.float32(p0[1])).astype(np.float32)
    o = (4 * (X.view(np.uint32) >> 31) + 2 * (Y.view(np.uint32) >> 31)
         + (np.abs(Y) > np.abs(X))).astype(np.int64)
    r2 = (X.astype(np.float64) ** 2 + Y.astype(np.float64) ** 2).astype(np.float32)
    tin, tout, tfar = b[:8][o], b[8:16][o], b[16]
    decided = (r2 < tin) | ((r2 > tout) & (r2 < tfar))
    return round(float(1.0 - decided.mean()), 5)


def margin_statistics(P, torch, o, V, Vt, Qt, Q, matrix, sample=1 << 22):
    """Float32 screen against binary64 on the first `sample` points (about
    1% of them within 1e-6 of an edge): the largest |M_hat - D| in units of
    u (alpha|X| + beta|Y| + gamma), u = 2^-24 (M_hat the float32 largest
    margin of the vector screen, pip_voronoi_max_margin; D the binary64 one
    of Algorithm 5, the oracle; alpha, beta, gamma the largest |A_i|, |B_i|,
    |C_i| of the screen table), the largest share of the band E it uses, and
    the share of points whose margin lies inside the band of the screen the
    launch takes (`matrix`: the matrix-core screen's wider band), i.e. the
    points sent to the binary64 recheck (estimated with the vector M_hat)."""
    S = int(min(sample, len(Q)))
    mh = P.pip_voronoi_max_margin(Vt, Qt[:S]).cpu().numpy().astype(np.float64)
    D = o.voronoi_max_margin(V, Q[:S].astype(np.float64))
    tab = P.pip_screen_table(Vt, 0, 0).cpu().numpy()
    ox, oy = np.float32(tab[0]), np.float32(tab[1])
    n4 = int(tab[6])
    rows = tab[12:12 + 4 * n4].reshape(n4, 4).astype(np.float64)
    X32 = Q[:S, 0] - ox  # float32 subtraction, as the screen
    Y32 = Q[:S, 1] - oy
    X = X32.astype(np.float64)
    Y = Y32.astype(np.float64)
    al, be, ga = np.abs(rows[:, 0]).max(), np.abs(rows[:, 1]).max(), np.abs(rows[:, 2]).max()
    err = np.abs(mh - D)
    scale = al * np.abs(X) + be * np.abs(Y) + ga

    def band(t, fold):
        full = (float(t[2]) * (X * X + Y * Y) + float(t[3]) * np.abs(X) + float(t[4]) * np.abs(Y)
                + float(t[5]))
        if not fold:
            return full
        # the vector screen's band: in 512-point chunks whose float32
        # |X| + |Y| are all within RQ, max(KA, KB) (|X| + |Y|) + KC
        s32 = (np.abs(X32) + np.abs(Y32)).astype(np.float64)
        lin = max(float(t[3]), float(t[4])) * s32 + float(t[5])
        ok = np.repeat((s32[: S // 512 * 512].reshape(-1, 512) <= float(t[8])).all(axis=1), 512)
        ok = np.concatenate([ok, np.zeros(S - ok.size, dtype=bool)])
        return np.where(ok, lin, full)
    E = band(tab, not matrix)
    Eb = band(P.pip_screen_table(Vt, 0, 1).cpu().numpy(), False) if matrix else E
    return {"sample_points": S,
            "max_err_u": round(float((err / scale).max() / 2.0 ** -24), 4),
            "max_err_over_band": round(float((err / E).max()), 4),
            "band_frac": round(float((~((mh < -Eb) | (mh > Eb))).mean()), 6)}


def _time(torch, stream, fn, reps=5, warm=1):
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def run_extras(P, W, torch, stream, check):
    """The other workload shapes: binary64 single polygon (all three tests),
    uneven batch (autotuned, graph-captured plan), all pairs, collision cost."""
    out = {}
    dev = "cuda"
    if check:
        from oracle import Oracle, pack_bits, unpack_bits
        o = Oracle()
    rng = np.random.default_rng(1234)

    # single polygon, 1e6 binary64 points, three tests
    V, Q = W.single_polygon_fp64()
    Vt, Qt = torch.from_numpy(V).to(dev), torch.from_numpy(Q).to(dev)
    lab = torch.empty((len(Q) + 31) // 32, dtype=torch.int32, device=dev)
    single = {"points": len(Q), "n": len(V), "point_dtype": "float64"}
    for name, fn, oname in (("voronoi", P.pip_voronoi, "voronoi"),
                            ("sign_of_offset", P.pip_sign_of_offset, "sign_of_offset"),
                            ("ray_crossing", P.pip_ray_crossing, "ray_crossing")):
        ms = _time(torch, stream, lambda: fn(Vt, Qt, lab), reps=20)
        entry = {"ms": round(ms, 4), "gtests_per_s": round(len(Q) / ms / 1e6, 2)}
        if check:
            got = lab.cpu().numpy().view(np.uint32)
            want = pack_bits(getattr(o, oname)(V, Q))
            entry["mismatches"] = int(np.unpackbits((got ^ want).view(np.uint8)).sum())
        single[name] = entry
    out["single_polygon_fp64"] = single
    print("[bench] single polygon done", file=sys.stderr, flush=True)

    # uneven batch
    B = W.uneven_batch()
    vo, Vb, po, Qb, lo = (torch.from_numpy(B.vtx_off).to(dev), torch.from_numpy(B.V).to(dev),
                          torch.from_numpy(B.pt_off).to(dev), torch.from_numpy(B.Q).to(dev),
                          torch.from_numpy(B.lbl_word_off).to(dev))
    plan = P.BatchedPlan(vo, Vb, po, Qb, lo)
    cfg, tuned_ms = plan.autotune(reps=3)
    ms = _time(torch, stream, plan.launch, reps=10)
    nt = B.num_tests
    entry = {"polygons": B.num_polygons, "tests": nt, "tile_shape": list(cfg),
             "autotune_ms": round(tuned_ms, 4), "graph_ms": round(ms, 4),
             "gtests_per_s": round(nt / ms / 1e6, 2),
             "hbm_frac": round(BYTES_PER_TEST * nt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if check:
        lab_b = plan.labels.cpu().numpy().view(np.uint32)
        bad = 0
        for k in sorted(rng.choice(B.num_polygons, 48, replace=False)):
            p0, p1 = B.pt_off[k], B.pt_off[k + 1]
            v0, v1 = B.vtx_off[k], B.vtx_off[k + 1]
            want = o.voronoi(B.V[v0:v1], B.Q[p0:p1].astype(np.float64))
            w0 = B.lbl_word_off[k]
            got = unpack_bits(lab_b[w0:w0 + (p1 - p0 + 31) // 32], p1 - p0)
            bad += int((got != want).sum())
        entry["mismatches_48_polygons"] = bad
    # chunks of 512 points whose labels are all outside: the only chunks an
    # early break (Section 5) taken by a whole wave could cut short
    lab_all = plan.labels.cpu().numpy().view(np.uint32)
    nch = zero = 0
    for k in range(B.num_polygons):
        s_k = int(B.pt_off[k + 1] - B.pt_off[k])
        w0 = int(B.lbl_word_off[k])
        for c in range(0, s_k, 512):
            nch += 1
            zero += int(not lab_all[w0 + c // 32: w0 + (min(s_k, c + 512) + 31) // 32].any())
    entry["chunks_all_outside"] = round(zero / max(nch, 1), 6)
    out["uneven_batch"] = entry
    plan.close()

    # a batch of 32-edge polygons: the per-edge screen (default) and the
    # radial pre-screen (reported apart), each in its own autotuned plan
    B32 = W.uneven_batch(n_lo=32, n_hi=32)
    t32 = [torch.from_numpy(a).to(dev) for a in (B32.vtx_off, B32.V, B32.pt_off, B32.Q,
                                                   B32.lbl_word_off)]
    e32 = {"polygons": B32.num_polygons, "tests": B32.num_tests}
    radial_min = int(P.get_option(P.PIP_OPT_RADIAL_MIN_EDGES))
    for key, rmin in (("graph_ms", radial_min), ("radial_graph_ms", 20)):
        P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, rmin)
        try:
            pl = P.BatchedPlan(*t32)
            pl.autotune(reps=3)
            e32[key] = round(_time(torch, stream, pl.launch, reps=10), 4)
            if check and key == "graph_ms":
                lab_b = pl.labels.cpu().numpy().view(np.uint32)
                bad = 0
                for k in sorted(rng.choice(B32.num_polygons, 16, replace=False)):
                    p0, p1 = B32.pt_off[k], B32.pt_off[k + 1]
                    v0, v1 = B32.vtx_off[k], B32.vtx_off[k + 1]
                    want = o.voronoi(B32.V[v0:v1], B32.Q[p0:p1].astype(np.float64))
                    w0 = B32.lbl_word_off[k]
                    got = unpack_bits(lab_b[w0:w0 + (p1 - p0 + 31) // 32], p1 - p0)
                    bad += int((got != want).sum())
                e32["mismatches_16_polygons"] = bad
            pl.close()
        finally:
            P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, radial_min)
    e32["gtests_per_s"] = round(B32.num_tests / e32["graph_ms"] / 1e6, 2)
    out["batch_n32"] = e32
    del t32
    del vo, Vb, po, Qb, lo, B
    torch.cuda.empty_cache()
    print("[bench] uneven batch done", file=sys.stderr, flush=True)

    # all pairs: 2048 poses x 131,072 points
    F = W.car_footprint()
    Qc = W.lidar_cloud()
    poses, cs = W.random_poses()
    Ft, Qct, pt, ct = (torch.from_numpy(F).to(dev), torch.from_numpy(Qc).to(dev),
                       torch.from_numpy(poses).to(dev), torch.from_numpy(cs).to(dev))
    Vw = P.pip_poses_to_polygons(Ft, pt, ct)
    labs = torch.empty((len(poses), (len(Qc) + 31) // 32), dtype=torch.int32, device=dev)
    cnts = torch.empty(len(poses), dtype=torch.int32, device=dev)

    def allpairs():
        P.pip_poses_to_polygons(Ft, pt, ct, out=Vw)
        P.pip_voronoi_allpairs(Vw, Qct, labels=labs, counts=cnts)
    ms = _time(torch, stream, allpairs, reps=10)
    nt = len(poses) * len(Qc)
    tfl = 4.0 * len(F) * nt / (ms * 1e-3) / 1e12
    entry = {"poses": len(poses), "points": len(Qc), "tests": nt, "ms": round(ms, 4),
             "gtests_per_s": round(nt / ms / 1e6, 1), "fp32_tflops": round(tfl, 2),
             "fp32_frac": round(tfl / FP32_VALU_PEAK_TFLOPS, 4)}
    if check:
        sel = np.sort(rng.choice(len(poses), 64, replace=False))
        bits, counts = o.allpairs(F, poses[sel, :2].astype(np.float64), cs[sel],
                                  Qc.astype(np.float64))
        got = labs.cpu().numpy().view(np.uint32)[sel]
        entry["mismatches_64_poses"] = int(np.unpackbits((got ^ bits).view(np.uint8)).sum())
    out["allpairs"] = entry
    # culled variant (a layer in front of the test, reported apart from the
    # dense row): (pose, wave) pairs whose bounding disk misses the wave's
    # points are skipped; labels and counts must equal the dense ones
    dense_l, dense_c = labs.clone(), cnts.clone()
    P.set_option(P.PIP_OPT_ALLPAIRS_CULL, 1)
    try:
        ms_c = _time(torch, stream, allpairs, reps=10)
        same = bool(torch.equal(labs, dense_l) and torch.equal(cnts, dense_c))
    finally:
        P.set_option(P.PIP_OPT_ALLPAIRS_CULL, 0)
    out["allpairs_culled"] = {"ms": round(ms_c, 4), "speedup_vs_dense": round(ms / ms_c, 2),
                              "dense_equivalent_gtests_per_s": round(nt / ms_c / 1e6, 1),
                              "labels_and_counts_equal_dense": same}
    # autotuned, graph-captured plan over the exact variants
    plan = P.AllpairsPlan(Vw, Qct)
    try:
        (cfg_c, cfg_p), tuned = plan.autotune(reps=5)
        ms_g = _time(torch, stream, plan.launch, reps=10)
        same = bool(torch.equal(plan.labels, dense_l) and torch.equal(plan.counts, dense_c))
    finally:
        plan.close()
    out["allpairs_plan"] = {"variant": {"cull": cfg_c, "pair": cfg_p}, "autotune_ms": round(tuned, 4),
                            "graph_ms": round(ms_g, 4),
                            "labels_and_counts_equal_dense": same}
    # antipodal pairing (the car is centrally symmetric: 4 pairs instead of
    # 8 edges), alone and with culling; labels and counts must equal the dense
    for key, cull in (("allpairs_paired", 0), ("allpairs_paired_culled", 1)):
        P.set_option(P.PIP_OPT_ALLPAIRS_PAIR, 1)
        P.set_option(P.PIP_OPT_ALLPAIRS_CULL, cull)
        try:
            ms_p = _time(torch, stream, allpairs, reps=10)
            same = bool(torch.equal(labs, dense_l) and torch.equal(cnts, dense_c))
        finally:
            P.set_option(P.PIP_OPT_ALLPAIRS_PAIR, 0)
            P.set_option(P.PIP_OPT_ALLPAIRS_CULL, 0)
        out[key] = {"ms": round(ms_p, 4), "speedup_vs_dense": round(ms / ms_p, 2),
                    "dense_equivalent_gtests_per_s": round(nt / ms_p / 1e6, 1),
                    "labels_and_counts_equal_dense": same}
    print("[bench] all pairs done", file=sys.stderr, flush=True)

    # coverage raster: 16384 x 16384 pixel points generated in the kernel
    # (no point array read: bound by the vector units)
    N = 16384
    rast = {"width": N, "height": N, "extent": [-1.5, 1.5]}
    for n in (8, 64):
        rr = np.random.default_rng(2007153852 + n)
        Vr = W.circle_polygon(n, 1.0, rr.uniform(-0.1, 0.1, 2), rr)
        Vrt = torch.from_numpy(Vr).to(dev)
        lab_r = P.pip_voronoi_raster(Vrt, -1.5, -1.5, 3.0 / N, 3.0 / N, N, N)
        ms_r = _time(torch, stream, lambda: P.pip_voronoi_raster(
            Vrt, -1.5, -1.5, 3.0 / N, 3.0 / N, N, N, labels=lab_r), reps=10)
        tfl = 4.0 * n * N * N / (ms_r * 1e-3) / 1e12
        e = {"ms": round(ms_r, 4), "gpixels_per_s": round(N * N / ms_r / 1e6, 1),
             "fp32_tflops": round(tfl, 2), "fp32_frac": round(tfl / FP32_VALU_PEAK_TFLOPS, 4)}
        radial_min = int(P.get_option(P.PIP_OPT_RADIAL_MIN_EDGES))
        if n >= 20 and not (radial_min > 0 and n >= radial_min):
            # the radial pre-screen (off by default), reported apart
            P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, 20)
            try:
                e["radial_ms"] = round(_time(torch, stream, lambda: P.pip_voronoi_raster(
                    Vrt, -1.5, -1.5, 3.0 / N, 3.0 / N, N, N, labels=lab_r), reps=10), 4)
            finally:
                P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, radial_min)
            lab_r = P.pip_voronoi_raster(Vrt, -1.5, -1.5, 3.0 / N, 3.0 / N, N, N, labels=lab_r)
        if radial_min > 0 and n >= radial_min:
            # the radial pre-screen decides most pixels from r2; the 4n flop
            # figure above is the per-edge work it replaces.  The per-edge
            # raster alone, for comparison:
            e["screen"] = "radial"
            e["per_edge_equivalent_tflops"] = e.pop("fp32_tflops")
            e["fp32_frac"] = None  # the 4n flop per pixel are not executed
            P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, 0)
            try:
                e["per_edge_ms"] = round(_time(torch, stream, lambda: P.pip_voronoi_raster(
                    Vrt, -1.5, -1.5, 3.0 / N, 3.0 / N, N, N, labels=lab_r), reps=10), 4)
            finally:
                P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, radial_min)
            lab_r = P.pip_voronoi_raster(Vrt, -1.5, -1.5, 3.0 / N, 3.0 / N, N, N, labels=lab_r)
        else:
            e["screen"] = "per_edge"
        # the paper's early break (Section 5) taken by whole 512-pixel
        # segments of the per-edge screen, reported apart (labels unchanged)
        if e["screen"] == "per_edge":
            base_lab = lab_r.clone()
            P.set_option(P.PIP_OPT_EARLY_EXIT, 1)
            try:
                e["early_exit_ms"] = round(_time(torch, stream, lambda: P.pip_voronoi_raster(
                    Vrt, -1.5, -1.5, 3.0 / N, 3.0 / N, N, N, labels=lab_r), reps=10), 4)
            finally:
                P.set_option(P.PIP_OPT_EARLY_EXIT, 0)
            e["early_exit_labels_equal"] = bool(torch.equal(lab_r, base_lab))
            # share of segments whose pixels are all outside (where it can fire)
            seg_words = lab_r.reshape(N, N // 512, 16)
            e["segments_all_outside"] = round(float((seg_words == 0).all(dim=2).float().mean()), 4)
            lab_r = base_lab
        if check:
            rows = np.sort(rr.choice(N, 64, replace=False))
            got = lab_r.cpu().numpy().view(np.uint32)[rows]
            want = np.stack([np.packbits(o.voronoi_raster(Vr, -1.5, -1.5 + int(j) * (3.0 / N),
                                                          3.0 / N, 3.0 / N, N, 1)[0],
                                         bitorder="little").view(np.uint32) for j in rows])
            e["mismatches_64_rows"] = int(np.unpackbits((got ^ want).view(np.uint8)).sum())
        rast[f"n{n}"] = e
    out["raster"] = rast
    print("[bench] raster done", file=sys.stderr, flush=True)

    # point location: 2^26 uniform points against a 256 x 256 jittered
    # partition (about 98k convex cells) through the grid index
    part = W.jittered_partition(256, 256, cell=1.0, split=0.5)
    Ql = torch.from_numpy(W.locate_points(part, 1 << 26)).to(dev)
    offl, Vl = torch.from_numpy(part.vtx_off).to(dev), torch.from_numpy(part.V).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    index = P.LocateIndex(offl, Vl)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    wsl = torch.empty(index.workspace_bytes(Ql.shape[0]), dtype=torch.uint8, device=dev)
    ids = index.locate(Ql, binned=False)
    ms_l = _time(torch, stream, lambda: index.locate(Ql, ids=ids, binned=False), reps=5)
    ids_b = index.locate(Ql, binned=True, workspace=wsl)
    ms_b = _time(torch, stream, lambda: index.locate(Ql, ids=ids_b, binned=True, workspace=wsl),
                 reps=5)
    cells, entries = index.info()
    e = {"polygons": len(part.vtx_off) - 1, "points": int(Ql.shape[0]), "cells": cells,
         "entries": entries, "build_ms": round(build_ms, 2), "ms": round(ms_l, 3),
         "gpoints_per_s": round(Ql.shape[0] / ms_l / 1e6, 2),
         "binned_ms": round(ms_b, 3), "binned_gpoints_per_s": round(Ql.shape[0] / ms_b / 1e6, 2),
         "binned_ids_equal": bool(torch.equal(ids, ids_b)),
         "hbm_frac_binned": round(12.0 * Ql.shape[0] / (ms_b * 1e-3) / 8.0e12, 4)}
    if check:
        sel = np.sort(rng.choice(Ql.shape[0], 4096, replace=False))
        want = o.locate(part.vtx_off, part.V, Ql.cpu().numpy()[sel].astype(np.float64))
        e["mismatches_4096_points"] = int((ids.cpu().numpy()[sel] != want).sum())
    index.close()
    out["locate"] = e
    print("[bench] locate done", file=sys.stderr, flush=True)

    # non-convex polygon: a 64-vertex star polygon as the union of the convex
    # pieces of the library's decomposition, 2^27 float32 points in
    # [-1.5, 1.5]^2 (1% within 1e-6 of an edge); every point meets every piece
    Vn = W.star_polygon(64)
    off_n, idx_n = P.convex_decompose(Vn, 64)
    mn = 1 << 27
    Qn = W.streaming_points(Vn, mn, seed_salt=77)
    Vnt, Qnt = torch.from_numpy(Vn).to(dev), torch.from_numpy(Qn).to(dev)
    offt, idxt = torch.from_numpy(off_n).to(dev), torch.from_numpy(idx_n).to(dev)
    labn = torch.empty((mn + 31) // 32, dtype=torch.int32, device=dev)
    stn = torch.empty(len(off_n) - 1, dtype=torch.int32, device=dev)
    wsn = torch.empty(max(P.pieces_workspace_bytes(len(off_n) - 1, len(idx_n)), 256),
                      dtype=torch.uint8, device=dev)
    ms_n = _time(torch, stream, lambda: P.pip_voronoi_pieces(Vnt, offt, idxt, Qnt, labels=labn,
                                                             status=stn, workspace=wsn), reps=10)
    rows = int(sum(((off_n[k + 1] - off_n[k] + 3) // 4) * 4 for k in range(len(off_n) - 1)))
    tfl = 4.0 * len(idx_n) * mn / (ms_n * 1e-3) / 1e12
    e = {"n": len(Vn), "pieces": len(off_n) - 1, "piece_edges": int(len(idx_n)),
         "padded_rows": rows, "points": mn, "ms": round(ms_n, 4),
         "gtests_per_s": round(mn / ms_n / 1e6, 2),
         "fp32_tflops_piece_edges": round(tfl, 2),
         "fp32_frac": round(tfl / FP32_VALU_PEAK_TFLOPS, 4),
         "hbm_frac": round(BYTES_PER_TEST * mn / (ms_n * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if check:
        got = unpack_bits(labn.cpu().numpy().view(np.uint32), mn)
        sel = np.sort(rng.choice(mn, 2_000_000, replace=False))
        want = o.voronoi_pieces(Vn, off_n, idx_n, Qn[sel].astype(np.float64))
        e["mismatches_2M_sample"] = int((got[sel] != want).sum())
    out["nonconvex"] = e
    del Qnt, Vnt, labn, wsn
    torch.cuda.empty_cache()
    print("[bench] non-convex done", file=sys.stderr, flush=True)

    # differentiable cost: 1024 trajectories x 64 poses x 65,536 points
    F32 = F.astype(np.float32)
    Qd = W.lidar_cloud(points_per_ring=1024, rings=64, config=5)
    tr = W.trajectories().reshape(-1, 3)
    F32t, Qdt, trt = (torch.from_numpy(F32).to(dev), torch.from_numpy(Qd).to(dev),
                      torch.from_numpy(tr).to(dev))
    ws = torch.empty(P.autograd.cost_workspace_bytes(len(F32), len(tr), len(Qd)),
                     dtype=torch.uint8, device=dev)
    ones = torch.ones(len(tr), dtype=torch.float32, device=dev)
    fwd_ms = _time(torch, stream, lambda: P.pip_cost_fwd(F32t, trt, Qdt, workspace=ws), reps=3)
    bwd_ms = _time(torch, stream, lambda: P.pip_cost_bwd(F32t, trt, Qdt, ones, workspace=ws),
                   reps=3)
    # culled variant (reported apart): results must be bit-identical
    c_dense = P.pip_cost_fwd(F32t, trt, Qdt, workspace=ws).clone()
    g_dense = [g.clone() for g in P.pip_cost_bwd(F32t, trt, Qdt, ones, workspace=ws)[:2]]
    P.set_option(P.PIP_OPT_COST_CULL, 1)
    try:
        fwd_c = _time(torch, stream, lambda: P.pip_cost_fwd(F32t, trt, Qdt, workspace=ws), reps=3)
        bwd_c = _time(torch, stream, lambda: P.pip_cost_bwd(F32t, trt, Qdt, ones, workspace=ws),
                      reps=3)
        c_cull = P.pip_cost_fwd(F32t, trt, Qdt, workspace=ws)
        g_cull = P.pip_cost_bwd(F32t, trt, Qdt, ones, workspace=ws)[:2]
        cull_same = bool(torch.equal(c_dense, c_cull) and torch.equal(g_dense[0], g_cull[0])
                         and torch.equal(g_dense[1], g_cull[1]))
    finally:
        P.set_option(P.PIP_OPT_COST_CULL, 0)
    out["cost_culled"] = {"fwd_ms": round(fwd_c, 4), "bwd_ms": round(bwd_c, 4),
                          "fwd_speedup_vs_dense": round(fwd_ms / fwd_c, 2),
                          "bwd_speedup_vs_dense": round(bwd_ms / bwd_c, 2),
                          "bit_identical_to_dense": cull_same}
    # antipodal pairs (the car footprint is centrally symmetric), alone and
    # with culling: results differ from the per-edge loop by rounding only
    for key, cull in (("cost_paired", 0), ("cost_paired_culled", 1)):
        P.set_option(P.PIP_OPT_COST_PAIR, 1)
        P.set_option(P.PIP_OPT_COST_CULL, cull)
        try:
            fwd_p = _time(torch, stream, lambda: P.pip_cost_fwd(F32t, trt, Qdt, workspace=ws), reps=3)
            bwd_p = _time(torch, stream,
                          lambda: P.pip_cost_bwd(F32t, trt, Qdt, ones, workspace=ws), reps=3)
            c_p = P.pip_cost_fwd(F32t, trt, Qdt, workspace=ws)
            diff = (c_p - c_dense).abs()
            rel = float((diff / (c_dense.abs() + 1e-3)).max())
        finally:
            P.set_option(P.PIP_OPT_COST_PAIR, 0)
            P.set_option(P.PIP_OPT_COST_CULL, 0)
        out[key] = {"fwd_ms": round(fwd_p, 4), "bwd_ms": round(bwd_p, 4),
                    "fwd_speedup_vs_dense": round(fwd_ms / fwd_p, 2),
                    "bwd_speedup_vs_dense": round(bwd_ms / bwd_p, 2),
                    "max_cost_diff_vs_dense": {"abs": float(diff.max()), "rel_to_cost_plus_1e-3": rel}}
    # autotuned, graph-captured plans (culling on or off, whichever is faster)
    plans = {}
    for key, bwd in (("fwd", False), ("bwd", True)):
        cp = P.CostPlan(F32t, trt, Qdt, backward=bwd, grad_cost=ones)
        try:
            (cc, _), tuned = cp.autotune(reps=2)
            plans[key] = {"cull": cc, "autotune_ms": round(tuned, 4),
                          "graph_ms": round(_time(torch, stream, cp.launch, reps=3), 4)}
        finally:
            cp.close()
    out["cost_plan"] = plans
    pairs = len(tr) * len(Qd)
    entry = {"poses": len(tr), "points": len(Qd), "pairs": pairs, "fwd_ms": round(fwd_ms, 3),
             "bwd_ms": round(bwd_ms, 3), "fwd_gpairs_per_s": round(pairs / fwd_ms / 1e6, 1),
             "bwd_gpairs_per_s": round(pairs / bwd_ms / 1e6, 1)}
    if check:
        c = P.pip_cost_fwd(F32t, trt, Qdt, workspace=ws).cpu().numpy()
        sel = np.sort(rng.choice(len(tr), 128, replace=False))
        want = o.cost(F32.astype(np.float64), tr[sel].astype(np.float64), Qd.astype(np.float64))
        rel = np.abs(c[sel] - want) / np.maximum(np.abs(want), 1e-6)
        entry["max_rel_err_128_poses"] = float(rel.max())
    out["cost"] = entry
    print("[bench] cost done", file=sys.stderr, flush=True)
    return out


def gpu_info(torch) -> dict:
    """Device name and the clocks rocm-smi reports right after the timed work
    (clocks are not pinned)."""
    info = {"name": torch.cuda.get_device_name(0)}
    try:
        import subprocess
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True,
                           timeout=30)
        data = json.loads(r.stdout) if r.returncode == 0 else {}
        card = next(iter(data.values()), {}) if isinstance(data, dict) else {}
        info["clocks"] = {k: v for k, v in card.items() if "clk" in k.lower()}
    except Exception as e:  # the clock query is informational only
        info["clocks"] = f"unavailable: {type(e).__name__}"
    return info


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--points", type=int, default=1 << 28, help="points per polygon")
    ap.add_argument("--cpu-sample", type=int, default=1 << 28,
                    help="points per polygon for the oracle baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched / all-pairs / cost / binary64 workloads")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 1 GiB device buffer 3 times (counter calibration)")
    ap.add_argument("--batch-run", action="store_true",
                    help="for counter runs: the 4096-polygon uneven batch as an autotuned, "
                         "graph-captured plan, then one more graph launch (the dispatch to read)")
    ap.add_argument("--traffic-run", action="store_true",
                    help="only one Voronoi launch per polygon size (for counter runs)")
    ap.add_argument("--ingest-counters", nargs=4,
                    metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="turn rocprofv3 FETCH_SIZE / WRITE_SIZE runs of --traffic-run and "
                         "--copy-probe into profiles/hbm_traffic.json")
    args = ap.parse_args()
    if args.ingest_counters:
        return ingest_counters(*args.ingest_counters)
    if args.copy_probe:
        import torch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 4}), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for {args.gpus}): the library has no "
              "multi-GPU launch; shard point ranges or polygons over processes instead",
              file=sys.stderr)
        return 2

    import torch
    import paper_2007_15385_amd as P
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    P.load_library()
    dev = torch.device("cuda:0")
    if args.batch_run:
        B = W.uneven_batch()
        t = [torch.from_numpy(a).to(dev) for a in (B.vtx_off, B.V, B.pt_off, B.Q, B.lbl_word_off)]
        plan = P.BatchedPlan(*t)
        cfg, ms = plan.autotune(reps=3)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        print(json.dumps({"batch_run": {"tests": B.num_tests, "tile_shape": list(cfg),
                                        "autotune_ms": round(ms, 4)}}), flush=True)
        plan.close()
        return 0
    torch.cuda.set_device(dev)
    m = int(args.points)

    # ---- inputs, resident in HBM -----------------------------------------
    t0 = time.time()
    polys, pts, labels = {}, {}, {}
    host_q = {}
    for n in NS:
        V = W.streaming_polygon(n)
        Q = W.streaming_points(V, m)
        polys[n] = torch.from_numpy(V).to(dev)
        pts[n] = torch.from_numpy(Q).to(dev)
        labels[n] = torch.empty((m + 31) // 32, dtype=torch.int32, device=dev)
        host_q[n] = (V, Q[: args.cpu_sample].copy())
        del Q
        print(f"[bench] inputs n={n} ready ({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    if args.traffic_run:
        for n in NS:
            P.pip_voronoi(polys[n], pts[n], labels[n])
        torch.cuda.synchronize()
        print(json.dumps({"traffic_run": list(NS)}), flush=True)
        return 0

    def step():
        for n in NS:
            P.pip_voronoi(polys[n], pts[n], labels[n])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---- timed region: K steps, per-launch HIP events on the launch stream --
    stream = torch.cuda.current_stream(dev)
    ev = {n: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)] for n in NS}
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for k in range(args.steps):
        for n in NS:
            a, b = ev[n][k]
            a.record(stream)
            P.pip_voronoi(polys[n], pts[n], labels[n])
            b.record(stream)
    end.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    ms_per_step = total_ms / args.steps
    per_n_all = {n: np.array([a.elapsed_time(b) for a, b in ev[n]]) for n in NS}
    per_n_ms = {n: float(per_n_all[n].mean()) for n in NS}
    tests_per_step = m * len(NS)
    value = tests_per_step / (ms_per_step * 1e-3) / 1e9
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)

    kernels = []
    for n in NS:
        t = per_n_ms[n] * 1e-3
        gbs = BYTES_PER_TEST * m / t / 1e9
        tfl = 4.0 * n * m / t / 1e12
        kernels.append({"n": n, "ms": round(per_n_ms[n], 4),
                        "ms_min": round(float(per_n_all[n].min()), 4),
                        "ms_median": round(float(np.median(per_n_all[n])), 4),
                        "ms_p90": round(float(np.percentile(per_n_all[n], 90)), 4),
                        "gtests_per_s": round(m / t / 1e9, 2),
                        "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                        "fp32_tflops": round(tfl, 2),
                        "fp32_frac": round(tfl / FP32_VALU_PEAK_TFLOPS, 4)})
    # which screen each polygon size takes: the radial pre-screen (if on for
    # this size) wins over the matrix cores, which win over the vector screen
    mfma_min = int(P.get_option(P.PIP_OPT_MFMA_MIN_EDGES))
    radial_min = int(P.get_option(P.PIP_OPT_RADIAL_MIN_EDGES))

    def screen_of(n):
        if radial_min > 0 and n >= radial_min:
            return "radial"
        return "mfma" if mfma_min > 0 and n >= mfma_min else "valu"

    for r in kernels:
        r["screen"] = screen_of(r["n"])
        if r["screen"] == "radial":
            r["radial_annulus_frac"] = annulus_fraction(P, torch, *host_q[r["n"]])
            # only the annulus points meet the 4n flop per-edge screen
            r["per_edge_equivalent_tflops"] = r.pop("fp32_tflops")
            r["fp32_frac"] = None
    if not args.no_cpu:
        # float32 margin error against binary64 and the share rechecked
        from oracle import Oracle
        o_stat = Oracle()
        for r in kernels:
            n = r["n"]
            V, Qs = host_q[n]
            r["margin_vs_binary64"] = margin_statistics(P, torch, o_stat, V, polys[n], pts[n], Qs,
                                                        r["screen"] == "mfma")
    dom = max(kernels, key=lambda r: r["ms"])
    # binding roofline of the dominant launch: bytes vs flops at peak
    t_hbm = BYTES_PER_TEST * m / (HBM_PEAK_GBS * 1e9)
    t_alu = 4.0 * dom["n"] * m / (FP32_VALU_PEAK_TFLOPS * 1e12)
    on_mfma = dom["screen"] == "mfma"
    if dom["screen"] == "radial":
        # a few operations per point; the per-edge screen runs on the annulus
        # points only, so the launch is priced by its bytes
        t_alu = 0.0
    if t_alu > t_hbm:
        # fp32 products on the matrix cores, or two fp32 fma per margin on the
        # vector units: both priced against the 157.3 TFLOP/s fp32 peak
        roof = {"bound": "mfma" if on_mfma else "alu", "achieved": dom["fp32_tflops"],
                "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": dom["fp32_frac"]}
    else:
        roof = {"bound": "hbm", "achieved": dom["hbm_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dom["hbm_frac"]}
    roof["kernel"] = (f"k_stream_mfma<voronoi,{64 if dom['n'] > 32 else 32}> n={dom['n']}"
                      if on_mfma else
                      f"k_stream32_radial n={dom['n']}" if dom["screen"] == "radial" else
                      f"k_stream32<voronoi> n={dom['n']}")
    roof["traffic"] = traffic_for(f"voronoi_f32_n{dom['n']}")
    roof["algorithmic_per_launch"] = ({"flop": 4.0 * dom["n"] * m}
                                      if roof["bound"] in ("alu", "mfma")
                                      else {"bytes": BYTES_PER_TEST * m})

    # ---- comparison kernels (outside the timed step) -----------------------
    def time_fn(fn, n, reps=3):
        fn(polys[n], pts[n], labels[n])
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn(polys[n], pts[n], labels[n])
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    # sign of offset and Voronoi timed back to back per polygon size, so that
    # both meet the same clock (under sustained load the part lowers its
    # clock within milliseconds; these launches follow the timed sweep)
    soo, vor_beside = {}, {}
    for n in NS:
        soo[n] = time_fn(P.pip_sign_of_offset, n)
        vor_beside[n] = time_fn(P.pip_voronoi, n)
    plain = {n: time_fn(P.pip_voronoi_fp32_plain, n) for n in NS}
    ray = {n: time_fn(P.pip_ray_crossing, n, reps=1) for n in NS}
    # the radial pre-screen (a culling layer in front of the test: points
    # between two radii per octant meet the per-edge screen, the others are
    # decided from their distance to p_0), reported apart from the dense
    # sweep; its labels must equal the dense ones word for word
    radial = {}
    for n in (16, 32, 64):
        dense = labels[n].clone()
        P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, 3)
        try:
            ms_r = time_fn(P.pip_voronoi, n)
            same = bool(torch.equal(labels[n], dense))
        finally:
            P.set_option(P.PIP_OPT_RADIAL_MIN_EDGES, radial_min)
        radial[str(n)] = {"ms": round(ms_r, 4), "speedup_vs_dense": round(per_n_ms[n] / ms_r, 2),
                          "dense_equivalent_gtests_per_s": round(m / ms_r / 1e6, 1),
                          "annulus_frac": annulus_fraction(P, torch, *host_q[n]),
                          "labels_equal_dense": same}
        del dense
    comparisons = {
        "voronoi_radial_prescreen": radial,
        "sign_of_offset_gtests_per_s": round(tests_per_step / (sum(soo.values()) * 1e-3) / 1e9, 2),
        "sign_of_offset_ms": {str(n): round(v, 4) for n, v in soo.items()},
        "voronoi_beside_sign_of_offset_gtests_per_s":
            round(tests_per_step / (sum(vor_beside.values()) * 1e-3) / 1e9, 2),
        "voronoi_beside_sign_of_offset_ms": {str(n): round(v, 4) for n, v in vor_beside.items()},
        "fp32_plain_gtests_per_s": round(tests_per_step / (sum(plain.values()) * 1e-3) / 1e9, 2),
        "fp32_plain_ms": {str(n): round(v, 4) for n, v in plain.items()},
        "ray_crossing_gtests_per_s": round(tests_per_step / (sum(ray.values()) * 1e-3) / 1e9, 2),
        "ray_crossing_ms": {str(n): round(v, 4) for n, v in ray.items()},
    }

    # ---- parity on a sample + oracle baseline ------------------------------
    mismatches = None
    plain_mismatches = None
    cpu = None
    if not args.no_cpu:
        from oracle import Oracle, pack_bits
        o = Oracle()
        S = int(min(args.cpu_sample, m))
        cpu_t = 0.0
        mismatches = 0
        plain_mismatches = 0
        ref_mismatches = {"sign_of_offset": 0, "ray_crossing": 0}

        def diff_bits(fn, n, want):
            fn(polys[n], pts[n], labels[n])
            got = labels[n][: (S + 31) // 32].cpu().numpy().view(np.uint32)
            return int(np.unpackbits((got ^ pack_bits(want)).view(np.uint8)).sum())
        for n in NS:
            V, Qs = host_q[n]
            Q64 = Qs.astype(np.float64)
            c0 = time.perf_counter()
            want = o.voronoi(V, Q64)
            cpu_t += time.perf_counter() - c0
            mismatches += diff_bits(P.pip_voronoi, n, want)
            plain_mismatches += diff_bits(P.pip_voronoi_fp32_plain, n, want)
            ref_mismatches["sign_of_offset"] += diff_bits(P.pip_sign_of_offset, n,
                                                          o.sign_of_offset(V, Q64))
            ref_mismatches["ray_crossing"] += diff_bits(P.pip_ray_crossing, n,
                                                        o.ray_crossing(V, Q64))
            del Q64, want
            print(f"[bench] parity n={n} done", file=sys.stderr, flush=True)
        threads = o.num_threads()
        # one thread on 1/64 of the sample
        s1 = max(S // 64, 1)
        o.set_num_threads(1)
        c0 = time.perf_counter()
        for n in NS:
            V, Qs = host_q[n]
            o.voronoi(V, Qs[:s1].astype(np.float64))
        t1 = time.perf_counter() - c0
        o.set_num_threads(threads)
        model = ""
        try:
            with open("/proc/cpuinfo") as fh:
                model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
        except OSError:
            pass
        cpu = {"value": round(S * len(NS) / cpu_t / 1e9, 5), "unit": "G tests/s",
               "cores": threads, "kind": "oracle",
               "sample": (f"all {S} points of each of the 6 polygons (the whole sweep, "
                          if S == m else f"first {S} points of each of the 6 polygons' arrays (")
                         + f"{S * len(NS)} tests), FP64 C oracle, OpenMP over points",
               "seconds": round(cpu_t, 2),
               "per_core_gtests_per_s": round(S * len(NS) / cpu_t / 1e9 / threads, 5),
               "single_thread_gtests_per_s": round(s1 * len(NS) / t1 / 1e9, 5),
               "single_thread_sample": f"first {s1} points of each polygon",
               "cpu_model": model, "host_cpus": os.cpu_count()}
        comparisons["fp32_plain_mismatches_on_sample"] = plain_mismatches
        comparisons["sign_of_offset_mismatches_on_sample"] = ref_mismatches["sign_of_offset"]
        comparisons["ray_crossing_mismatches_on_sample"] = ref_mismatches["ray_crossing"]

    extras = {} if args.no_extras else run_extras(P, W, torch, stream, not args.no_cpu)
    gpu = gpu_info(torch)

    out = {
        "metric": "G point-polygon tests/s (Voronoi, every edge of every point: certified "
                  "float32 screen + binary64 recheck, labels bit-identical to the FP64 oracle)",
        "value": round(value, 2),
        "unit": "G tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "streaming sweep: convex polygons with n = 3,4,8,16,32,64 "
                               "vertices (radius 1, centre in [-0.1,0.1]^2), each against "
                               f"{m} float32 points in [-1.5,1.5]^2, 1% within 1e-6 of an edge",
                   "points_per_polygon": m, "polygons": list(NS), "point_dtype": "float32"},
        "mismatches_on_sample": mismatches,
        "roofline": roof,
        "kernels": kernels,
        "comparisons": comparisons,
        "cpu_baseline": cpu,
        "gpu": gpu,
        "workloads": extras,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
