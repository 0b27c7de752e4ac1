"""CPU tests of libblest's host side through the C-ABI: exported symbols, argument
and graph validation, and parity of the host-side hot-path steps with the oracle -
BVSS construction (Section 2.1), Algorithm 1, RCM, the social-like test, the
statistics of Sections 2.2/2.2.1 and the static eager/lazy rule.  Handles are built
host-only (device = -1), so no GPU is touched."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import inputs
import paper_2512_21967_amd as blest
from oracle import bvss as obvss
from oracle import reorder as oreorder
from tests import families

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def host_graph(g, **kw):
    kw.setdefault("device", -1)
    return blest.Graph(g, **kw)


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "blest.h")).read()
    declared = set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(blest_\w+)\s*\(", header, re.M))
    assert "blest_build" in declared and "blest_bfs_multi" in declared
    L = ctypes.CDLL(blest.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(L, name), f"{name} missing from libblest.so"
    assert declared == set(blest.EXPORTED_SYMBOLS)


def test_status_strings():
    L = blest.lib()
    for code in range(9):
        assert L.blest_status_string(code)


def raw_build(n, rp, col, opt=None):
    L = blest.lib()
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(rp, np.uint32)
    col = np.ascontiguousarray(col if len(col) else [0], np.uint32)
    o = opt or blest.default_options()
    if opt is None:
        o.device = -1
    rc = L.blest_build(n, int(rp[-1]) if len(rp) else 0, blest._p32(rp), blest._p32(col), ctypes.byref(o),
                       ctypes.byref(h))
    if rc == 0:
        L.blest_destroy(h)
    return rc


def test_graph_validation_errors():
    assert raw_build(3, [0, 1, 2, 2], [1, 2]) == 0
    assert raw_build(3, [0, 2, 1, 2], [1, 2]) == 2            # row_ptr not monotone
    assert raw_build(3, [0, 1, 2, 2], [1, 3]) == 2            # column out of range
    assert raw_build(3, [1, 1, 2, 2], [1, 2]) == 2            # row_ptr[0] != 0
    L = blest.lib()
    h = ctypes.c_void_p()
    rp = np.array([0, 1], np.uint32)
    col = np.array([0], np.uint32)
    o = blest.default_options()
    o.device = -1
    assert L.blest_build(0, 0, blest._p32(rp), blest._p32(col), ctypes.byref(o), ctypes.byref(h)) == 1
    assert L.blest_build(1, 2 ** 32, blest._p32(rp), blest._p32(col), ctypes.byref(o), ctypes.byref(h)) == 3
    assert L.blest_build(1, 0, None, None, ctypes.byref(o), ctypes.byref(h)) == 1
    assert L.blest_build(1, 0, blest._p32(rp), blest._p32(col), ctypes.byref(o), None) == 1
    for field, bad in (("sigma", 12), ("slots", 3), ("window", 12), ("reorder", 9), ("update", -1), ("block", 100),
                       ("group", 3), ("blocks_per_cu", 3), ("ranges", 3), ("ranges", 64)):
        o = blest.default_options()
        o.device = -1
        setattr(o, field, bad)
        assert raw_build(2, [0, 1, 1], [1], o) == 1, field


def test_self_loops_and_duplicates_dropped():
    g = host_graph(types_graph(4, [0, 2, 4, 4, 4], [0, 1, 1, 1]), reorder="none")
    assert g.stats()["m"] == 1


def types_graph(n, rp, col):
    class G:
        pass
    x = G()
    x.n, x.row_ptr, x.col = n, np.array(rp, np.uint32), np.array(col, np.uint32)
    return x


def test_bfs_calls_on_host_only_handle():
    gr, _ = families.path(10)
    g = host_graph(gr)
    L = blest.lib()
    assert L.blest_bfs(g.handle, 10, ctypes.c_void_p(1), None, None) == 1     # source out of range
    assert L.blest_bfs(g.handle, 0, None, None, None) == 1                    # no output
    assert L.blest_bfs(g.handle, 0, ctypes.c_void_p(1), None, None) == 7      # host-only handle
    src = np.array([0, 1], np.uint32)
    assert L.blest_bfs_multi(g.handle, blest._p32(src), 0, ctypes.c_void_p(1), None) == 1
    assert L.blest_bfs_multi(g.handle, blest._p32(src), 65, ctypes.c_void_p(1), None) == 1
    bad = np.array([0, 10], np.uint32)
    assert L.blest_bfs_multi(g.handle, blest._p32(bad), 2, ctypes.c_void_p(1), None) == 1
    assert L.blest_bfs_multi(g.handle, blest._p32(src), 2, ctypes.c_void_p(1), None) == 7
    hs = (ctypes.c_void_p * 1)(g.handle.value)
    outs = (ctypes.c_void_p * 1)(1)
    one = np.array([0], np.uint32)
    assert L.blest_bfs_many(hs, blest._p32(one), 1, outs, None) == 7
    assert L.blest_bfs_many(hs, blest._p32(one), 0, outs, None) == 1


# ---------------------------------------------------------------------------
# BVSS structure parity with the oracle
# ---------------------------------------------------------------------------

def relabelled(gr, new_id):
    return inputs.relabel(gr, new_id) if not np.array_equal(new_id, np.arange(gr.n)) else gr


def check_row_range_cut(sid, row, mask, n_sets, tau, range_len, rp, v2r, beg, rows, mvals, vss_range):
    """The library's optional row-range cut is a layout choice, not the paper's
    partition, so it is checked by its properties: read in order, a set's VSSs hold
    exactly the set's slices (the oracle's, by definition); every VSS holds 1..tau
    slices whose rows lie in the VSS's own range; a VSS ends early only where its set
    ends or the next slice falls in another range."""
    bounds = np.searchsorted(sid, np.arange(n_sets + 1), side="left")
    assert rp[0] == 0 and len(rp) == n_sets + 1
    for s in range(n_sets):
        vs = range(rp[s], rp[s + 1])
        assert all(v2r[v] == s for v in vs)
        lo, hi = bounds[s], bounds[s + 1]
        if hi == lo:
            assert len(vs) == 0
            continue
        a, b = beg[rp[s]], beg[rp[s + 1]]
        np.testing.assert_array_equal(rows[a:b], row[lo:hi])
        np.testing.assert_array_equal(mvals[a:b], mask[lo:hi])
        for v in vs:
            r = rows[beg[v]:beg[v + 1]]
            assert 1 <= len(r) <= tau
            assert np.all(r // range_len == vss_range[v])
            if len(r) < tau and v + 1 < rp[s + 1]:
                assert rows[beg[v + 1]] // range_len != vss_range[v]


def check_bvss_against_oracle(gr, g, sigma, slots):
    new_id = g.export("new_id")
    assert sorted(new_id.tolist()) == list(range(gr.n))
    h = relabelled(gr, new_id)
    sid, row, mask = obvss.slices(h, sigma)
    n_sets = obvss.num_slice_sets(h.n, sigma)
    tau = 64 * slots
    st = g.stats()
    rp = g.export("real_ptrs")
    v2r = g.export("virtual_to_real")
    beg = g.export("vss_begin")
    rows = g.export("row_ids")
    masks = g.export("masks")
    mb = sigma // 8
    mvals = np.zeros(len(rows), np.uint64)
    for b in range(mb):
        mvals |= masks[b::mb].astype(np.uint64) << np.uint64(8 * b)
    assert beg[0] == 0 and beg[-1] == len(rows) == len(sid)
    if st["nranges"] > 1:
        check_row_range_cut(sid, row, mask, n_sets, tau, st["range_len"], rp, v2r, beg, rows, mvals,
                            g.export("vss_range"))
    else:
        part = obvss.vss_partition(sid, row, mask, n_sets, tau)
        np.testing.assert_array_equal(rp, part["realPtrs"])
        np.testing.assert_array_equal(v2r, part["virtualToReal"])
        for v, (r, m) in enumerate(part["groups"]):
            np.testing.assert_array_equal(rows[beg[v]:beg[v + 1]], r)
            np.testing.assert_array_equal(mvals[beg[v]:beg[v + 1]], m)
        assert not np.any(g.export("vss_range"))
    assert st["num_slices"] == len(sid) and st["num_vss"] == len(v2r) and st["tau"] == tau
    assert st["compression"] == pytest.approx(obvss.compression_ratio(h.nnz, len(sid), sigma))
    # the update-scheme policy reads the divergence of the ordering before the hub sort
    o = relabelled(gr, g.export("order_id"))
    osid, orow, omask = obvss.slices(o, sigma)
    paper_groups = obvss.vss_partition(osid, orow, omask, n_sets, 32 * (32 // sigma))["groups"]
    assert st["u_div_paper"] == pytest.approx(obvss.update_divergence(paper_groups, 32), rel=1e-9, abs=1e-9)
    native_groups = [(rows[beg[v]:beg[v + 1]], None) for v in range(len(v2r))]
    assert st["u_div_native"] == pytest.approx(obvss.update_divergence(native_groups, 64), rel=1e-9, abs=1e-9)
    assert st["nranges"] >= 1 and st["range_len"] % 32 == 0
    assert st["bvss_bytes_table3"] == obvss.bvss_bytes_table3(len(sid), len(v2r), n_sets, sigma)


@pytest.mark.parametrize("sigma,slots", [(8, 1), (8, 4), (16, 2), (32, 1), (8, 8)])
def test_bvss_matches_oracle_rmat(sigma, slots):
    gr = inputs.rmat_workload(11, 16, seed=sigma + slots, permute_seed=2)
    g = host_graph(gr, sigma=sigma, slots=slots, reorder="none")
    check_bvss_against_oracle(gr, g, sigma, slots)


def test_bvss_matches_oracle_directed_and_ragged():
    rng = np.random.default_rng(3)
    for n in (1, 7, 63, 65, 200, 1001):
        m = n * 5
        gr = inputs.from_arcs(n, rng.integers(0, n, m), rng.integers(0, n, m), False)
        g = host_graph(gr, sigma=8, slots=1, reorder="none")
        check_bvss_against_oracle(gr, g, 8, 1)


@pytest.mark.parametrize("ranges", [2, 8, 32])
def test_bvss_row_ranges_match_oracle(ranges):
    gr = inputs.rmat_workload(12, 16, seed=ranges, permute_seed=5)
    g = host_graph(gr, sigma=8, slots=2, reorder="none", update="lazy", ranges=ranges)
    st = g.stats()
    assert st["nranges"] == ranges and st["range_len"] * ranges >= gr.n
    check_bvss_against_oracle(gr, g, 8, 2)
    assert st["num_vss"] > host_graph(gr, sigma=8, slots=2, reorder="none", update="lazy").stats()["num_vss"]


def test_auto_ranges_keep_one_range():
    gr = inputs.rmat_workload(20, 8, seed=1, permute_seed=2)
    lazy = host_graph(gr, reorder="none", update="lazy").stats()
    eager = host_graph(gr, reorder="none", update="eager").stats()
    assert lazy["nranges"] == 1 and eager["nranges"] == 1
    assert lazy["range_len"] >= gr.n and lazy["num_vss"] == eager["num_vss"]


@pytest.mark.parametrize("reorder", ["compression", "bandwidth"])
def test_bvss_matches_oracle_after_reordering(reorder):
    gr = inputs.rmat_workload(10, 8, seed=5, permute_seed=1) if reorder == "compression" else \
        inputs.grid_workload(40, 0.9, seed=2, permute_seed=6)
    g = host_graph(gr, sigma=8, slots=2, reorder=reorder, window=256)
    check_bvss_against_oracle(gr, g, 8, 2)


# ---------------------------------------------------------------------------
# Orderings and the static policy
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_jaccard_windows_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    sigma = [8, 16, 8, 32, 8, 8][seed]
    w = sigma * int(rng.integers(2, 9))
    if seed % 2 == 0:
        gr = inputs.rmat_workload(8, 8, seed=seed, permute_seed=seed + 10)
    else:
        n = int(rng.integers(20, 300))
        m = n * int(rng.integers(1, 6))
        gr = inputs.from_arcs(n, rng.integers(0, n, m), rng.integers(0, n, m), bool(seed % 3))
    g = host_graph(gr, sigma=sigma, window=w, reorder="compression", prepass="off")
    np.testing.assert_array_equal(g.export("order_id"), oreorder.jaccard_with_windows(gr, sigma, w))
    if not g.stats()["hubs_sorted"]:
        np.testing.assert_array_equal(g.export("new_id"), g.export("order_id"))


def test_jaccard_windows_matches_oracle_hand_cases():
    for adj, n, sigma, w in (({0: [4, 5], 1: [6], 2: [4], 3: [5]}, 8, 8, 8),
                             ({0: [4], 1: [5, 6], 2: [4, 5, 6], 3: [4, 8, 9, 10]}, 16, 8, 8)):
        src = [u for u, vs in adj.items() for _ in vs]
        dst = [v for vs in adj.values() for v in vs]
        gr = inputs.from_arcs(n, src, dst, False)
        g = host_graph(gr, sigma=sigma, window=w, reorder="compression", hubs="off", prepass="off")
        np.testing.assert_array_equal(g.export("new_id"), oreorder.jaccard_with_windows(gr, sigma, w))


@pytest.mark.parametrize("case", ["grid", "rmat", "union", "directed", "isolated"])
def test_rcm_matches_oracle(case):
    rng = np.random.default_rng(1)
    if case == "grid":
        gr = inputs.grid_workload(23, 0.9, seed=5, permute_seed=2)
    elif case == "rmat":
        gr = inputs.rmat_workload(9, 4, seed=3, permute_seed=4)
    elif case == "union":
        gr = inputs.relabel(families.disjoint_union_paths(9, 14)[0], inputs.permutation(23, 3))
    elif case == "directed":
        gr = inputs.from_arcs(150, rng.integers(0, 150, 300), rng.integers(0, 150, 300), False)
    else:
        gr = inputs.from_arcs(30, [1, 5, 9], [2, 6, 10], True)
    g = host_graph(gr, reorder="bandwidth")
    np.testing.assert_array_equal(g.export("order_id"), oreorder.rcm(gr))


def hub_sorted_labels(gr, order_id, sigma, cpos):
    """The hub sort by its definition: the sigma-groups inside complete 32-vertex
    words, ranked by summed in-degree (largest first, ties in order), fill words in
    rank order; ranked words take the positions 0..cpos-1 of every 64-word chunk
    first (round t gives chunk c position (t + c) mod cpos), then the other
    positions in order."""
    spw = 32 // sigma
    fw = gr.n // 32
    fg = fw * spw
    indeg = np.bincount(gr.col.astype(np.int64), minlength=gr.n)
    lab_deg = np.zeros(gr.n, np.int64)
    lab_deg[order_id] = indeg
    w = lab_deg[:fg * sigma].reshape(fg, sigma).sum(axis=1) if fg else np.zeros(0, np.int64)
    ranked = sorted(range(fg), key=lambda g: (-w[g], g))
    chunks = -(-fw // 64)
    cp = min(cpos, 64)
    slots = [c * 64 + (t + c) % cp for t in range(cp) for c in range(chunks) if c * 64 + (t + c) % cp < fw]
    first = set(slots)
    slots += [q for q in range(fw) if q not in first]
    new_group = np.empty(fg, np.int64)
    for r, g in enumerate(ranked):
        new_group[g] = slots[r // spw] * spw + r % spw
    out = order_id.astype(np.int64).copy()
    move = out < fg * sigma
    out[move] = new_group[out[move] // sigma] * sigma + out[move] % sigma
    return out


@pytest.mark.parametrize("case", ["rmat-compression", "rmat-none", "ragged", "directed", "small-cache", "no-cache"])
def test_hub_sort_follows_its_definition(case):
    rng = np.random.default_rng(4)
    if case == "rmat-compression":
        gr, kw = inputs.rmat_workload(10, 8, seed=5, permute_seed=1), dict(reorder="compression", window=256)
    elif case == "rmat-none":
        gr, kw = inputs.rmat_workload(10, 16, seed=2), dict(reorder="none", sigma=16)
    elif case == "ragged":  # n not a multiple of sigma: the partial group stays last
        src = (rng.pareto(1.5, 6000) * 10).astype(np.int64) % 1001
        gr, kw = inputs.from_arcs(1001, src, rng.integers(0, 1001, 6000), True), dict(reorder="none")
    elif case == "directed":
        gr, kw = inputs.from_arcs(300, rng.integers(0, 300, 2000) ** 2 % 300, rng.integers(0, 300, 2000), False), \
            dict(reorder="none")
    elif case == "small-cache":  # 512 words in 8 chunks, 256 cached words: the first 32 of each chunk
        gr, kw = inputs.rmat_workload(14, 8, seed=9, permute_seed=3), dict(reorder="none", lds_kib=1)
    else:
        gr, kw = inputs.rmat_workload(14, 8, seed=9, permute_seed=3), dict(reorder="none", lds_kib=None)
    sigma = kw.get("sigma", 8)
    off = host_graph(gr, hubs="off", **kw)
    on = host_graph(gr, hubs="on", **kw)
    assert on.stats()["hubs_sorted"] == 1 and off.stats()["hubs_sorted"] == 0
    np.testing.assert_array_equal(on.export("order_id"), off.export("new_id"))
    cpos = on.stats()["hub_cpos"]
    assert cpos == {"small-cache": 32, "no-cache": 0}.get(case, 64)
    np.testing.assert_array_equal(on.export("new_id"), hub_sorted_labels(gr, on.export("order_id"), sigma, cpos))
    # same slice sets and masks, so the same slice count and compression
    a, b = on.stats(), off.stats()
    assert a["num_slices"] == b["num_slices"] and a["compression"] == b["compression"]
    assert a["u_div_paper"] == pytest.approx(b["u_div_paper"], rel=1e-12)
    check_bvss_against_oracle(gr, on, sigma, on.stats()["tau"] // 64)


def test_social_like_and_auto_policy():
    cases = [inputs.rmat(12, 16, seed=1), inputs.grid(50, 50, 0.9, seed=1), families.star(300)[0],
             families.path(300)[0], inputs.from_arcs(20, [], [], False)]
    for gr in cases:
        g = host_graph(gr, window=64)
        st = g.stats()
        social = oreorder.is_social_like(gr)
        assert bool(st["social_like"]) == social
        assert st["reorder_used"] == ("compression" if social else "bandwidth")
        lazy = social and st["u_div_paper"] > 25000
        assert st["update_used"] == ("lazy" if lazy else "eager")


def test_auto_update_rule_threshold():
    # Section 4: a graph smaller than ~50K vertices cannot exceed the 25,000 threshold
    g = host_graph(inputs.rmat_workload(12, 16, seed=1, permute_seed=3), reorder="none")
    assert g.stats()["update_used"] == "eager"
    # random labels at scale 19 spread each VSS column over ~29K IDs: lazy
    g = host_graph(inputs.rmat_workload(19, 16, seed=1, permute_seed=3), reorder="none")
    st = g.stats()
    assert st["u_div_paper"] > 25000 and st["update_used"] == "lazy"


def test_footprint_and_model_bytes():
    gr = inputs.rmat(10, 8, seed=2)
    g = host_graph(gr, reorder="none")
    f0, f1, f8, f64 = (g.footprint(k) for k in (0, 1, 8, 64))
    assert f0 == g.stats()["bvss_device_bytes"] and 0 < f1 < f8 < f64
    lv = np.full(gr.n, -1, np.int32)
    lv[0] = 0
    b_one = g.model_bytes(lv)
    lv[:] = 0
    b_all = g.model_bytes(lv)
    assert 4 * gr.n < b_one < b_all


@pytest.mark.parametrize("update", ["eager", "lazy", "adaptive"])
def test_model_bytes_single_source_formula(update):
    """k = 1 algorithmic bytes: for every iteration i = 1 .. max level + 1 and every
    slice set holding a vertex of level i - 1, its unpadded slices at 4 + sigma/8
    bytes, its sigma/8-byte frontier chunk and 8 bytes per VSS; 2 n/8 bytes of
    visited bitmaps per lazily run iteration (adaptive: queue >= eager_max); 4n bytes
    of level initialisation and 4 bytes per reached vertex.  Restated here from the
    exported arrays and the oracle's levels."""
    import oracle
    gr = inputs.rmat_workload(11, 8, seed=3, permute_seed=4)
    g = host_graph(gr, reorder="compression", window=256, update=update, eager_max=7)
    st = g.stats()
    sig = st["sigma"]
    new_id = g.export("new_id")
    rp = g.export("real_ptrs").astype(np.int64)
    vb = g.export("vss_begin").astype(np.int64)
    for s in (0, 5, 77):
        lv = oracle.bfs(gr, int(inputs.sources(gr, seed=s, k=1)[0]))
        lv_new = np.full(gr.n, -1, np.int64)
        lv_new[new_id] = lv
        sets = np.arange(gr.n) // sig
        total = 0
        maxl = int(lv.max())
        for i in range(1, maxl + 2):
            active = np.unique(sets[lv_new == i - 1])
            active = active[rp[active + 1] > rp[active]]
            slices = vb[rp[active + 1]] - vb[rp[active]]
            nvss = rp[active + 1] - rp[active]
            total += int(np.sum(slices * (4 + sig // 8) + sig // 8 + 8 * nvss))
            queued = int(nvss.sum())
            if update == "lazy" or (update == "adaptive" and queued >= 7):
                total += 2 * ((gr.n + 7) // 8)
        total += 4 * gr.n + 4 * int(np.sum(lv >= 0))
        assert g.model_bytes(lv) == total, (update, s)


def test_traffic_record_hash_scope():
    """The traffic record's hash covers the files that build the single-source
    kernel; every one of them exists, and the hash changes with their content."""
    from paper_2512_21967_amd import profsum
    for f in profsum.SINGLE_SOURCE_FILES:
        assert os.path.exists(os.path.join(profsum.CSRC, f)), f
    a = profsum.kernel_source_hash(profsum.SINGLE_SOURCE_FILES)
    assert a == profsum.kernel_source_hash(list(reversed(profsum.SINGLE_SOURCE_FILES)))
    assert a != profsum.kernel_source_hash(profsum.SINGLE_SOURCE_FILES[:-1])


SHINGLE_SEED = 0x243F6A8885A308D3  # the library's default seed


@pytest.mark.parametrize("seed", range(4))
def test_shingle_prepass_matches_oracle(seed):
    from oracle import prepass as oprepass
    rng = np.random.default_rng(40 + seed)
    k = [1, 2, 3, 8][seed]
    if seed % 2 == 0:
        gr = inputs.rmat_workload(8, 8, seed=seed, permute_seed=seed + 5)
    else:
        n = int(rng.integers(30, 200))
        m = n * int(rng.integers(1, 5))
        gr = inputs.from_arcs(n, rng.integers(0, n, m), rng.integers(0, n, m), bool(seed % 3))
    hseed = SHINGLE_SEED if seed < 2 else int(rng.integers(1 << 62))
    sigma, w = 8, 8 * int(rng.integers(2, 6))
    g = host_graph(gr, sigma=sigma, window=w, reorder="compression", hubs="off", prepass="shingle", shingles=k,
                   shingle_seed=hseed)
    assert g.stats()["prepass_used"] == 1
    np.testing.assert_array_equal(g.export("prepass_id"), oprepass.shingle_order(gr, k, hseed))
    np.testing.assert_array_equal(g.export("order_id"), oprepass.prepass_then_windows(gr, k, hseed, sigma, w))


def test_shingle_prepass_defaults_and_switches():
    gr = inputs.rmat_workload(9, 8, seed=3, permute_seed=4)
    auto = host_graph(gr, reorder="compression")
    on = host_graph(gr, reorder="compression", prepass="shingle")
    off = host_graph(gr, reorder="compression", prepass="off")
    assert auto.stats()["prepass_used"] == 1 and on.stats()["prepass_used"] == 1 and off.stats()["prepass_used"] == 0
    # default windows: 4096 after the pre-pass, 65536 without it
    assert auto.stats()["window_used"] == 4096 and off.stats()["window_used"] == 65536
    np.testing.assert_array_equal(auto.export("order_id"), on.export("order_id"))
    # two min-hashes and the seed 0x243F6A8885A308D3 by default
    from oracle import prepass as oprepass
    np.testing.assert_array_equal(on.export("prepass_id"), oprepass.shingle_order(gr, 2, SHINGLE_SEED))
    np.testing.assert_array_equal(on.export("order_id"), oprepass.prepass_then_windows(gr, 2, SHINGLE_SEED, 8, 4096))
    explicit = host_graph(gr, reorder="compression", window=64)
    assert explicit.stats()["window_used"] == 64
    np.testing.assert_array_equal(off.export("prepass_id"), np.arange(gr.n))
    np.testing.assert_array_equal(off.export("order_id"), oreorder.jaccard_with_windows(gr, 8, 1 << 16))
    # RCM and the given labels never run the pre-pass
    for r in ("bandwidth", "none"):
        h = host_graph(gr, reorder=r, prepass="shingle")
        assert h.stats()["prepass_used"] == 0 and h.stats()["window_used"] == 0
        np.testing.assert_array_equal(h.export("prepass_id"), np.arange(gr.n))
    with pytest.raises(blest.BlestError):
        host_graph(gr, prepass="shingle", shingles=9)


def test_shingle_prepass_groups_planted_twins():
    """Twin groups scattered by a permutation end up one slice set each when the
    pre-pass runs first; Algorithm 1 alone, with windows of one slice set, cannot
    gather them (the oracle's pin of the same case)."""
    sigma, groups, fan = 8, 64, 6
    src, dst = [], []
    for gi in range(groups):
        for j in range(sigma):
            for t in range(fan):
                src.append(gi * sigma + j)
                dst.append(groups * sigma + gi * fan + t)
    n = groups * (sigma + fan)
    gr = inputs.relabel(inputs.from_arcs(n, src, dst, False), inputs.permutation(n, 9))
    on = host_graph(gr, reorder="compression", window=sigma, prepass="shingle", hubs="off")
    off = host_graph(gr, reorder="compression", window=sigma, prepass="off", hubs="off")
    assert on.stats()["num_slices"] == groups * fan
    assert off.stats()["num_slices"] > groups * fan
