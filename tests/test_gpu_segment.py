"""The source-segmented layout (pr_segment_count, pr_prepare_segmented) and pr_pull on it, through
the C ABI.

* The layout is integer work and is compared bit for bit with a plain numpy construction from its
  definition (pairs = runs of one row's entries whose sources share a segment of seg_len ids, cut
  every 1024 entries of the row; pair CSR listed segment by segment, rows ascending; merge CSR
  listing every row's pairs in segment order).
* Solves on it keep the float64 bar of tests/parity.py against the oracle (1e-12 L1 after the
  same number of updates, traces, iteration counts with the tie rule), and the mixed and
  float32-only bars; they are bitwise repeatable; with option "segmented" = 0 the same buffer
  gives the plain update.
"""
import ctypes

import numpy as np
import pytest

import graphgen as gg
from parity import check_fp64_result, check_mixed_result

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PAIR_MAX = 1024


@pytest.fixture(scope="module")
def pr():
    import paper_2108_02997_amd as pr
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return pr


@pytest.fixture(scope="module")
def ctx(pr):
    c = pr.Context(0)
    yield c
    c.close()


class PrepPart(ctypes.Structure):
    _fields_ = [("desc_off", ctypes.c_int64), ("hub_off", ctypes.c_int64), ("tile", ctypes.c_int32),
                ("rows", ctypes.c_int32), ("ndesc", ctypes.c_int32), ("nslots", ctypes.c_int32),
                ("nhubs", ctypes.c_int32), ("pad", ctypes.c_int32)]


class SegLayout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("pairs", "poff_off", "moff_off", "mpos_off", "sidx_off", "part_off",
                                              "scan_off", "temp_off", "cub_off", "total")] + \
               [("pair_part", PrepPart), ("merge_part", PrepPart), ("tsort_off", ctypes.c_int64),
                ("tsort_bytes", ctypes.c_int64)]


class PrepHeader(ctypes.Structure):
    """The library's prep header as laid out in the buffer (internal.h)."""
    _fields_ = [("magic", ctypes.c_int32), ("version", ctypes.c_int32), ("N", ctypes.c_int64), ("E", ctypes.c_int64),
                ("seg", ctypes.c_int32), ("pad", ctypes.c_int32), ("scan_off", ctypes.c_int64),
                ("part", PrepPart * 2), ("seg_len", ctypes.c_int32), ("pad2", ctypes.c_int32), ("sl", SegLayout)]


def expected_layout(g, seg_len):
    """The segmented layout from its definition (numpy, row order first)."""
    off = g.off.astype(np.int64)
    idx = g.idx.astype(np.int64)
    E = g.E
    rows = np.repeat(np.arange(g.N, dtype=np.int64), np.diff(off))
    rel = np.arange(E, dtype=np.int64) - off[rows]
    seg = idx // seg_len
    start = (rel % PAIR_MAX == 0)
    start[1:] |= seg[1:] != seg[:-1]
    q_start = np.flatnonzero(start)                     # row-order pairs
    P = q_start.size
    q_len = np.diff(np.append(q_start, E))
    q_seg = seg[q_start]
    perm = np.argsort(q_seg, kind="stable")              # segment-major position -> row-order pair
    mpos = np.empty(P, dtype=np.int64)
    mpos[perm] = np.arange(P)
    poff = np.concatenate([[0], np.cumsum(q_len[perm])])
    sidx = np.concatenate([idx[q_start[q]:q_start[q] + q_len[q]] for q in perm]) if P else np.zeros(0, np.int64)
    first_pair = np.cumsum(start) - 1                    # row-order pair of every entry
    moff = np.empty(g.N + 1, dtype=np.int64)
    moff[g.N] = P
    nonempty = np.diff(off) > 0
    moff[:g.N][nonempty] = first_pair[off[:-1][nonempty]]
    # an empty row's pairs start where the next pairs start
    for v in range(g.N - 1, -1, -1):
        if not nonempty[v]:
            moff[v] = moff[v + 1]
    return P, poff, sidx, moff, mpos


def read_layout(dg):
    raw = dg.prep.cpu().numpy()
    h = PrepHeader.from_buffer_copy(raw[:ctypes.sizeof(PrepHeader)].tobytes())
    sl = h.sl

    def arr(at, n):
        return raw[at:at + 4 * n].view(np.int32).astype(np.int64)
    P = sl.pairs
    return h, P, arr(sl.poff_off, P + 1), arr(sl.sidx_off, dg.E), arr(sl.moff_off, dg.N + 1), arr(sl.mpos_off, P)


POS_BITS = 11


def read_tiles(dg):
    """The pair partition's tiles: entry starts (ndesc + 1 of them), each tile's base (descriptor w,
    -1 for a tile in pair order) and the raw index words."""
    raw = dg.prep.cpu().numpy()
    h = PrepHeader.from_buffer_copy(raw[:ctypes.sizeof(PrepHeader)].tobytes())
    sl = h.sl
    nd = sl.pair_part.ndesc
    desc = raw[sl.pair_part.desc_off:sl.pair_part.desc_off + 16 * (nd + 1)].view(np.int32).reshape(nd + 1, 4)
    words = raw[sl.sidx_off:sl.sidx_off + 4 * dg.E].view(np.uint32).astype(np.int64)
    return desc[:, 1].astype(np.int64), desc[:nd, 3].astype(np.int64), words


def unpack_tiles(starts, base, words):
    """Per entry: its tile, its source and its position in the tile's pair order."""
    tile = np.repeat(np.arange(starts.size - 1), np.diff(starts))
    b = base[tile]
    packed = b >= 0
    src = np.where(packed, b + (words >> POS_BITS), words)
    pos = np.where(packed, words & ((1 << POS_BITS) - 1), np.arange(words.size) - starts[tile])
    return tile, src, pos


def segmented(pr, ctx, g, seg_len):
    dg = pr.DeviceGraph.from_host(g)
    dg.prepare_segmented(ctx, seg_len=seg_len)
    return dg


def hub_graph(N=6000, seed=4):
    rng = np.random.default_rng(seed)
    src, dst = [], []
    for v, deg in ((0, 5000), (3, 2500), (7, 1100), (11, 300)):
        src.extend(rng.choice(N, size=deg, replace=False).tolist())
        dst.extend([v] * deg)
    src.extend(rng.integers(0, N, 30000).tolist())
    dst.extend(rng.integers(0, N, 30000).tolist())
    return gg.from_edges(N, src, dst)


def multi_graph(N=4000, seed=6):
    # every row draws 20 sources, with replacement, from a pool of 600: duplicate edges, so equal
    # sources within rows and within tiles (their order in a source-ordered tile is pair order);
    # vertices outside the pool are dangling
    rng = np.random.default_rng(seed)
    dst = np.repeat(np.arange(N), 20)
    src = rng.integers(0, 600, dst.size)
    return gg.from_edges(N, src, dst, dedupe=False, drop_self_loops=False)


GRAPHS = {
    "rmat13": lambda: gg.rmat(13, seed=31),
    "er_c1": gg.workload_c1,
    "hubs": hub_graph,
    "multi": multi_graph,
}


@pytest.mark.parametrize("name,seg_len", [("rmat13", 256), ("rmat13", 1024), ("rmat13", 3 * 1024 + 7),
                                          ("rmat13", 8192), ("er_c1", 512), ("er_c1", 3000), ("hubs", 256),
                                          ("hubs", 4096), ("multi", 256), ("multi", 300)])
def test_layout_matches_definition(pr, ctx, name, seg_len):
    g = GRAPHS[name]()
    check_layout(g, segmented(pr, ctx, g, seg_len), seg_len)


def check_layout(g, dg, seg_len):
    """The prep buffer's segmented layout against its definition; returns the tiles' bases."""
    P, poff, sidx, moff, mpos = expected_layout(g, seg_len)
    h, Pd, poff_d, sidx_d, moff_d, mpos_d = read_layout(dg)
    assert h.seg_len == seg_len and Pd == P == dg.seg_pairs
    np.testing.assert_array_equal(poff_d, poff)
    np.testing.assert_array_equal(moff_d, moff)
    np.testing.assert_array_equal(mpos_d, mpos)
    assert h.sl.pair_part.nhubs == 0 and int(np.diff(poff).max()) <= PAIR_MAX
    # a tile whose sources span fewer than 2^21 ids lists them in source order (ties in pair order),
    # each word packing the source less the tile's smallest one (descriptor w) and the entry's
    # pair-order position; any other tile holds the definition's entries as they are
    starts, base, words = read_tiles(dg)
    assert starts[0] == 0 and starts[-1] == g.E and np.all(np.diff(starts) > 0)
    assert np.all(np.diff(starts) < 1 << POS_BITS)           # a tile's positions fit the word
    tile, src, pos = unpack_tiles(starts, base, words)
    np.testing.assert_array_equal(src, sidx[starts[tile] + pos])
    np.testing.assert_array_equal(np.sort(starts[tile] + pos), np.arange(g.E))   # positions: a permutation
    first = starts[:-1]
    span = np.maximum.reduceat(sidx, first) - np.minimum.reduceat(sidx, first)
    np.testing.assert_array_equal(base >= 0, span < 1 << (32 - POS_BITS))
    np.testing.assert_array_equal(base[base >= 0], np.minimum.reduceat(sidx, first)[base >= 0])
    sorted_tiles = (base >= 0)[tile]
    order = np.lexsort((pos, src, tile))                     # tile, then source, then position
    np.testing.assert_array_equal(order[sorted_tiles[order]], np.flatnonzero(sorted_tiles))
    return base


def test_wide_tiles_stay_in_pair_order(pr, ctx):
    # 3M vertices, 2^21-id segments: tiles within a segment are packed in source order, tiles
    # that straddle the boundary may span 2^21 ids or more and keep their pair order; both kinds
    # are summed exactly as the oracle's rows
    g = gg.er(3_000_000, 2.0, seed=13)
    dg = segmented(pr, ctx, g, 1 << 21)
    base = check_layout(g, dg, 1 << 21)
    print("tiles %d, in pair order %d" % (base.size, int((base < 0).sum())), flush=True)
    assert (base >= 0).any() and (base < 0).any()
    res = pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=1, max_iter=500, trace=True)
    check_fp64_result(g, res["ranks"].cpu().numpy(), res["iterations"], res["converged"], 0.85, 1e-10, 1, 500,
                      gpu_trace=res["trace"].cpu().numpy())


@pytest.mark.parametrize("name,seg_len", [("rmat13", 256), ("rmat13", 2048), ("rmat13", 1500), ("er_c1", 1024),
                                          ("hubs", 512), ("multi", 256)])
def test_fp64_parity_every_norm(pr, ctx, name, seg_len):
    g = GRAPHS[name]()
    dg = segmented(pr, ctx, g, seg_len)
    for norm in (1, 2, 3):
        for alpha, tau in ((0.85, 1e-10), (0.5, 1e-6), (0.99, 1e-8)):
            res = pr.pull(ctx, dg, alpha=alpha, tau=tau, norm=norm, max_iter=500, trace=True)
            check_fp64_result(g, res["ranks"].cpu().numpy(), res["iterations"], res["converged"], alpha, tau, norm,
                              500, gpu_trace=res["trace"].cpu().numpy())


def test_alpha_one_and_zero(pr, ctx):
    g = gg.rmat(12, seed=5)
    dg = segmented(pr, ctx, g, 256)
    for alpha in (0.0, 1.0):
        res = pr.pull(ctx, dg, alpha=alpha, tau=1e-9, norm=1, max_iter=300, trace=True)
        check_fp64_result(g, res["ranks"].cpu().numpy(), res["iterations"], res["converged"], alpha, 1e-9, 1, 300,
                          gpu_trace=res["trace"].cpu().numpy())


def test_mixed_and_fp32_only(pr, ctx):
    g = gg.rmat(14, seed=8)
    dg = segmented(pr, ctx, g, 1024)
    for norm in (1, 3):
        res = pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=norm, max_iter=500, precision=pr.PR_MIXED)
        assert res["converged"] and res["fp32_iters"] >= 1
        check_mixed_result(g, res["ranks"].cpu().numpy(), res["err"], 0.85, 1e-10, norm)
        res = pr.pull(ctx, dg, alpha=0.85, tau=1e-7, norm=norm, max_iter=500, precision=pr.PR_FP32)
        check_mixed_result(g, res["ranks"].cpu().numpy(), res["err"], 0.85, 1e-7, norm, fp32_only=True)


def test_bitwise_repeatable_and_plain_switch(pr, ctx):
    g = gg.rmat(14, seed=9)
    dg = segmented(pr, ctx, g, 512)
    a = pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=1)
    b = pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=1)
    assert torch.equal(a["ranks"], b["ranks"]) and a["iterations"] == b["iterations"]
    ctx.set_option("segmented", 0)
    try:
        c = pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=1)
    finally:
        ctx.set_option("segmented", 1)
    assert abs(c["iterations"] - a["iterations"]) <= 1
    assert pr.l1_distance(ctx, a["ranks"], c["ranks"]) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tiles_per_xcd_or_round_robin(pr, ctx, precision):
    # the tile order of either step only regroups the norm partials: the same ranks bit for bit
    # after a fixed number of updates, norms equal up to the order of their sums, oracle parity
    g = gg.rmat(15, seed=10)
    dg = segmented(pr, ctx, g, 1024)
    prec = pr.PR_FP64 if precision == "fp64" else pr.PR_FP32
    its = 25 if precision == "fp64" else 12  # float32: well above its rounding floor
    runs = {}
    for sx, mx in ((1, 1), (0, 1), (1, 0), (0, 0)):
        ctx.set_option("seg_xcd", sx)
        ctx.set_option("merge_xcd", mx)
        try:
            runs[sx, mx] = pr.pull(ctx, dg, alpha=0.85, tau=0.0, norm=1, max_iter=its, trace=True, precision=prec)
        finally:
            ctx.set_option("seg_xcd", 1)
            ctx.set_option("merge_xcd", 0)
    for key, r in runs.items():
        assert r["iterations"] == its and torch.equal(r["ranks"], runs[1, 1]["ranks"]), key
        np.testing.assert_allclose(r["trace"].cpu().numpy(), runs[1, 1]["trace"].cpu().numpy(), rtol=1e-6, atol=0)
    if precision == "fp64":
        check_fp64_result(g, runs[1, 1]["ranks"].cpu().numpy(), 25, False, 0.85, 0.0, 1, 25,
                          gpu_trace=runs[1, 1]["trace"].cpu().numpy())
    for key in ("seg_xcd", "merge_xcd"):
        with pytest.raises(pr.PrError):
            ctx.set_option(key, 2)
    # any grid of the per-segment step (a multiple of 8 or not) gives the same partial sums
    for grid in (8, 1000, 24):
        ctx.set_option("seg_grid", grid)
        try:
            r = pr.pull(ctx, dg, alpha=0.85, tau=0.0, norm=1, max_iter=its, precision=prec)
        finally:
            ctx.set_option("seg_grid", 0)
        assert torch.equal(r["ranks"], runs[1, 1]["ranks"]), grid
    for bad in (-1, 16385):
        with pytest.raises(pr.PrError):
            ctx.set_option("seg_grid", bad)


@pytest.mark.parametrize("pair_mid_deg", [0, 8, 1024])
def test_pair_threshold(pr, ctx, pair_mid_deg):
    # every pair summed by a wave (0), mixed (8), every pair by one lane (1024): oracle parity
    g = hub_graph()
    dg = segmented(pr, ctx, g, 512)
    ctx.set_option("pair_mid_deg", pair_mid_deg)
    try:
        res = pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=2, max_iter=500, trace=True)
    finally:
        ctx.set_option("pair_mid_deg", 256)
    check_fp64_result(g, res["ranks"].cpu().numpy(), res["iterations"], res["converged"], 0.85, 1e-10, 2, 500,
                      gpu_trace=res["trace"].cpu().numpy())
    with pytest.raises(pr.PrError):
        ctx.set_option("pair_mid_deg", 1025)


def test_given_start_and_edgeless(pr, ctx):
    g = gg.rmat(12, seed=12)
    dg = segmented(pr, ctx, g, 256)
    rng = np.random.default_rng(3)
    init = rng.random(g.N)
    init /= init.sum()
    res = pr.pull(ctx, dg, alpha=0.85, tau=1e-9, norm=2, init=torch.from_numpy(init).cuda(), trace=True)
    check_fp64_result(g, res["ranks"].cpu().numpy(), res["iterations"], res["converged"], 0.85, 1e-9, 2, 500,
                      init=init, gpu_trace=res["trace"].cpu().numpy())
    # no edges: the plain partitions alone (every vertex dangling, 1/N after one update)
    e = gg.from_edges(50, [], [])
    de = segmented(pr, ctx, e, 256)
    r = pr.pull(ctx, de, alpha=0.85, tau=1e-12, norm=1)
    assert r["iterations"] == 1 and float((r["ranks"] - 1.0 / 50).abs().max()) < 1e-17


def test_count_and_arguments(pr, ctx):
    g = gg.rmat(10, seed=2)
    dg = pr.DeviceGraph.from_host(g)
    ws = torch.empty(16384, dtype=torch.uint8, device="cuda")
    pairs = ctypes.c_int64()
    lib = ctx.lib
    for seg_len in (256, 1000, 1 << 20):
        assert lib.pr_segment_count(ctx.handle, ctx.stream, dg.off.data_ptr(), dg.idx.data_ptr(), g.N, g.E, seg_len,
                                    ws.data_ptr(), ws.numel(), ctypes.byref(pairs)) == 0
        assert pairs.value == expected_layout(g, seg_len)[0]
    assert lib.pr_segment_count(ctx.handle, ctx.stream, dg.off.data_ptr(), dg.idx.data_ptr(), g.N, g.E, 255,
                                ws.data_ptr(), ws.numel(), ctypes.byref(pairs)) == pr._lib.PR_EINVAL
    assert lib.pr_segment_count(ctx.handle, ctx.stream, dg.off.data_ptr(), dg.idx.data_ptr(), g.N, g.E, 1024,
                                ws.data_ptr(), 100, ctypes.byref(pairs)) == pr._lib.PR_ENOMEM
    P = expected_layout(g, 1024)[0]
    nbytes = lib.pr_segment_bytes(ctx.handle, g.N, g.E, 1024, P)
    assert nbytes > lib.pr_prep_bytes(g.N, g.E)
    assert lib.pr_segment_bytes(ctx.handle, g.N, g.E, 1024, g.E + 1) == 0
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    # a pair count that is not the graph's is refused before the layout is built
    assert lib.pr_prepare_segmented(ctx.handle, ctx.stream, dg.off.data_ptr(), dg.idx.data_ptr(), g.N, g.E, 1024,
                                    P - 1, buf.data_ptr(), nbytes) == pr._lib.PR_EINVAL
    assert lib.pr_prepare_segmented(ctx.handle, ctx.stream, dg.off.data_ptr(), dg.idx.data_ptr(), g.N, g.E, 1024,
                                    P, buf.data_ptr(), nbytes - 1) == pr._lib.PR_ENOMEM


def test_scale22_fp64_against_oracle(pr, ctx):
    g = gg.rmat(22, edge_factor=16, seed=22)
    dg = segmented(pr, ctx, g, 1 << 18)
    print("scale 22: N %d E %d pairs %d (%.3f E)" % (g.N, g.E, dg.seg_pairs, dg.seg_pairs / g.E), flush=True)
    res = pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=1, max_iter=500, trace=True)
    ref = check_fp64_result(g, res["ranks"].cpu().numpy(), res["iterations"], res["converged"], 0.85, 1e-10, 1, 500,
                            gpu_trace=res["trace"].cpu().numpy())
    print("scale 22 segmented: %d updates (oracle %d)" % (res["iterations"], ref["iterations"]), flush=True)


def test_autotune_segmented_layout(pr, tmp_path):
    # with the segmented layout in the prep buffer the autotuner also times the segmented update
    # (pair threshold x per-segment grid x merge tile order), keeps its choice for the graph and
    # writes it to the tune file; solves on the tuned settings keep oracle parity
    import os
    tune = tmp_path / "tune.txt"
    os.environ["PRPULL_TUNE_FILE"] = str(tune)
    try:
        c = pr.Context(0)
    finally:
        del os.environ["PRPULL_TUNE_FILE"]
    try:
        g = gg.rmat(15, seed=41)
        dg = segmented(pr, c, g, 2048)
        t = dg.autotune(c)
        assert t["seg_candidates"] == 16
        assert t["pair_mid_deg"] in (64, 128, 256, 512) and t["seg_grid"] > 0 and t["merge_xcd"] in (0, 1)
        assert 0.0 < t["best_seg_us"] <= t["default_seg_us"]
        seg_lines = [ln.split() for ln in tune.read_text().splitlines() if ln.startswith("seg ")]
        assert len(seg_lines) == 1 and seg_lines[0][9] == "2048"
        assert [int(x) for x in seg_lines[0][10:]] == [t["pair_mid_deg"], t["seg_grid"], t["merge_xcd"]]
        for norm in (1, 3):
            res = pr.pull(c, dg, alpha=0.85, tau=1e-10, norm=norm, trace=True)
            check_fp64_result(g, res["ranks"].cpu().numpy(), res["iterations"], res["converged"], 0.85, 1e-10, norm,
                              500, gpu_trace=res["trace"].cpu().numpy())
        # a context reading the file solves the same way
        os.environ["PRPULL_TUNE_FILE"] = str(tune)
        try:
            c2 = pr.Context(0)
        finally:
            del os.environ["PRPULL_TUNE_FILE"]
        try:
            a = pr.pull(c, dg, alpha=0.85, tau=0.0, norm=1, max_iter=20)
            b = pr.pull(c2, dg, alpha=0.85, tau=0.0, norm=1, max_iter=20)
            assert torch.equal(a["ranks"], b["ranks"])
        finally:
            c2.close()
        # a plain prep has no segmented stage
        dp = pr.DeviceGraph.from_host(g).prepare(c)
        t2 = dp.autotune(c)
        assert t2["seg_candidates"] == 0 and t2["pair_mid_deg"] == 0 and t2["best_seg_us"] == 0.0
    finally:
        c.close()
