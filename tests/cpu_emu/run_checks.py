"""Run parity checks against the CPU-emulated build of the library --
TEST INFRASTRUCTURE.  Must run in a process started with libasan preloaded
(see tests/test_cpu_emulation.py).  Exits nonzero on the first mismatch."""
import ctypes
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402
import paper_1209_6007_amd as sbc  # noqa: E402
from tests.helpers import assert_bc_close  # noqa: E402


def use_emulated(path):
    L = ctypes.CDLL(path)
    for name, (args, res) in sbc._SIGS.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    sbc._lib = L


def check(name, fn):
    print(f"-- {name}", flush=True)
    fn()


def main(which):
    use_emulated(os.path.join(ROOT, "_build", "emu", "libshatterbc_emu.so"))
    # one resident block per launch and 4-wave batch blocks keep the
    # thread-per-lane emulation fast; the kernels' logic is the same
    ctx = sbc.Context(0, {"team_wg_waves": 4, "slots": 1, "batch_wg_waves": 4})
    if "single" in which:
        def single():
            # per-source levels, path counts and dependencies written by the
            # dump variant of each traversal kernel
            g = gg.decorated_random(40, 0.08, 10, 6, 3, 2000)
            reach, ident = gg.random_attributes(g.n, 3000)
            tctx = sbc.Context(0, {"team_wg_waves": 4, "slots": 0, "batch_wg_waves": 4, "team_count": 2})
            for r, k in ((None, None), (reach, ident)):
                for s in (0, g.n // 2, g.n - 1):
                    d, sg, dl = sbc.sbc_single_source(ctx.h, g.n, g.row_ptr, g.col, s, r, k)
                    od, osg, odl = oracle.single_source(g.n, g.row_ptr, g.col, s, r, k)
                    np.testing.assert_array_equal(d, od)
                    np.testing.assert_array_equal(sg, osg)
                    m = od > 0
                    np.testing.assert_allclose(dl[m], odl[m], rtol=1e-9)
                src = np.array([0, 5, g.n - 1, 17, 3], np.int32)
                for kernel, c in ((3, ctx), (4, tctx), (5, ctx)):
                    d, sg, dl = sbc.sbc_sources_state(c.h, g.n, g.row_ptr, g.col, src, kernel, r, k)
                    for row, s in enumerate(src):
                        od, osg, odl = oracle.single_source(g.n, g.row_ptr, g.col, int(s), r, k)
                        np.testing.assert_array_equal(d[row], od)
                        np.testing.assert_array_equal(sg[row], osg)
                        m = od > 0
                        np.testing.assert_allclose(dl[row][m], odl[m], rtol=1e-9)
                        assert np.all(dl[row][od <= 0] == 0)
                    print(f"   kernel {kernel} weighted={r is not None} ok", flush=True)
            tctx.close()
        check("single source", single)
    full = os.environ.get("SBC_EMU_FULL") == "1"
    if "pieces" in which:
        def pieces():
            cases = [(5, 3), (5, 5), (65, 5), (70, 3), (130, 3)]
            if full:
                cases = [(n, k) for n in (3, 5, 64, 65, 130, 700) for k in (3, 5) if not (k == 5 and n > 256)]
            for n, kernel in cases:
                r = gg.rng(n * 7 + kernel)
                g = gg.erdos_renyi(n, min(0.9, 6.0 / max(n - 1, 1)), int(r.integers(1 << 30)))
                reach, ident = gg.random_attributes(n, int(r.integers(1 << 30)), rmax=5, kmax=3)
                for rr, kk in (((None, None), (reach, ident)) if full or n < 10 else ((reach, ident),)):
                    want = oracle.bc_weighted(g.n, g.row_ptr, g.col, rr, kk)
                    got = sbc.sbc_piece_bc(ctx.h, g.n, g.row_ptr, g.col, rr, kk, kernel=kernel)
                    assert_bc_close(got, want, 1e-9, f"piece n={n} kernel={kernel}")
                print(f"   n={n} kernel={kernel} ok", flush=True)
            # the batch kernel's 64-lane row layout (the compact layout is the default)
            rctx = sbc.Context(0, {"team_wg_waves": 4, "slots": 1, "batch_wg_waves": 4, "batch_compact": 0})
            g = gg.erdos_renyi(130, 0.05, 77)
            reach, ident = gg.random_attributes(g.n, 78, rmax=5, kmax=3)
            want = oracle.bc_weighted(g.n, g.row_ptr, g.col, reach, ident)
            assert_bc_close(sbc.sbc_piece_bc(rctx.h, g.n, g.row_ptr, g.col, reach, ident, kernel=3), want, 1e-9,
                            "row layout")
            rctx.close()
            print("   n=130 kernel=3 row layout ok", flush=True)
        check("piece kernels", pieces)
    if "whole" in which:
        def whole():
            graphs = [("grid8", gg.grid_deleted(side=8, seed=9)), ("rmat6", gg.rmat_decorated(scale=6, seed=3)),
                      ("decorated", gg.decorated_random(30, 0.1, 8, 5, 3, 11)),
                      ("empty", gg.csr_from_edges(5, [], [])), ("path2", gg.path(2))]
            if full:
                graphs += [("ba2100", gg.ba_pendant_triangles()), ("grid16", gg.grid_deleted(side=16, seed=9)),
                           ("rmat8", gg.rmat_decorated(scale=8, seed=3))]
            for name, g in graphs:
                want = oracle.bc(g)
                sbc.sbc_context_set_param(ctx.h, "order_plain", 1)
                assert_bc_close(sbc.betweenness(g.n, g.row_ptr, g.col, mode="plain", ctx=ctx), want, 1e-9,
                                f"{name}/plain ordered")
                assert_bc_close(sbc.betweenness(g.n, g.row_ptr, g.col, mode="compressed", ops="odai", ctx=ctx), want,
                                1e-9, f"{name}/odai")
                sbc.sbc_context_set_param(ctx.h, "order_plain", 0)
                # default routing, then every piece on the batch kernel, with
                # and without the pair path
                # (deep_min_levels 2 sends every piece deeper than two levels
                # to the deep class's own launch, in 4-wave workgroups)
                for wave_max, pairs, deep in ((256, 16, 64), (0, 64, 64), (0, 0, 64), (0, 16, 2)):
                    sbc.sbc_context_set_param(ctx.h, "wave_max_vertices", wave_max)
                    sbc.sbc_context_set_param(ctx.h, "batch_pairs", pairs)
                    sbc.sbc_context_set_param(ctx.h, "deep_min_levels", deep)
                    sbc.sbc_context_set_param(ctx.h, "deep_wg_waves", 4)
                    for mode in ("plain", "compressed"):
                        got = sbc.betweenness(g.n, g.row_ptr, g.col, mode=mode, ctx=ctx)
                        assert_bc_close(got, want, 1e-9, f"{name}/{mode}/wave_max={wave_max}/pairs={pairs}/deep={deep}")
                sbc.sbc_context_set_param(ctx.h, "wave_max_vertices", 256)
                sbc.sbc_context_set_param(ctx.h, "batch_pairs", 16)
                sbc.sbc_context_set_param(ctx.h, "deep_min_levels", 64)
                # side vertices (Algorithm 3 items) on every kernel class
                for ops in ("odasi", "dasi"):
                    for wave_max in (256, 0):
                        sbc.sbc_context_set_param(ctx.h, "wave_max_vertices", wave_max)
                        assert_bc_close(sbc.betweenness(g.n, g.row_ptr, g.col, mode="compressed", ops=ops, ctx=ctx),
                                        want, 1e-9, f"{name}/{ops}/wave_max={wave_max}")
                sbc.sbc_context_set_param(ctx.h, "wave_max_vertices", 256)
                # deterministic mode: per-item areas, the same bits twice
                d1 = sbc.betweenness(g.n, g.row_ptr, g.col, mode="compressed+deterministic", ops="odai", ctx=ctx)
                d2 = sbc.betweenness(g.n, g.row_ptr, g.col, mode="compressed+deterministic", ops="odai", ctx=ctx)
                assert np.array_equal(d1, d2), name
                assert_bc_close(d1, want, 1e-9, f"{name}/deterministic")
                print(f"   {name} n={g.n} ok", flush=True)
        check("whole graphs", whole)

        def copybw():
            gb = sbc.sbc_copy_bandwidth(ctx.h, 1 << 16, 2)
            assert gb > 0
        check("copy calibration", copybw)

        def phases():
            g = gg.rmat_decorated(scale=7, seed=3)
            pctx = sbc.Context(0, {"team_wg_waves": 4, "slots": 1, "batch_wg_waves": 4, "profile_phases": 1, "wave_max_vertices": 0})
            G = sbc.Graph(g.n, g.row_ptr, g.col)
            G.preprocess("dai")
            plan = sbc.sbc_plan_create(pctx.h, G.h, sbc.SBC_COMPRESSED)
            sbc.sbc_plan_execute(plan)
            sbc.sbc_plan_sync(plan)
            ph = sbc.sbc_plan_phase_profile(plan)
            assert_bc_close(sbc.sbc_plan_result(plan, g.n), oracle.bc(g), 1e-9, "profiled run")
            sbc.sbc_plan_destroy(plan)
            assert ph["items"] >= 1 and ph["levels"] >= 1 and ph["entries"] >= ph["items"], ph
            print("   phases", {k: round(v, 3) for k, v in ph.items()}, flush=True)
        check("phase timers", phases)
    if "hubs" in which:
        def hubs():
            # a vertex with more arcs than the batch kernel's split threshold
            n = 1300
            r = gg.rng(5)
            u = np.concatenate([np.zeros(1200, np.int64), r.integers(1, n, 600)])
            v = np.concatenate([np.arange(1, 1201), r.integers(1, n, 600)])
            g2 = gg.csr_from_edges(n, u, v)
            src = np.arange(0, 70, dtype=np.int32)
            want = oracle.bc_plain(g2.n, g2.row_ptr, g2.col, sources=src)
            G = sbc.Graph(g2.n, g2.row_ptr, g2.col)
            got = sbc.sbc_betweenness_sources(ctx.h, G.h, src)
            assert_bc_close(got, want, 1e-9, "hub rows")
        check("split rows", hubs)
    if "team" in which:
        def team():
            # every piece on the team kernel.  Emulated XCD k hosts blocks 2k and
            # 2k+1: 2 teams of 2 workgroups on one XCD each; one team of 3 over
            # two XCDs (uneven ranks, agent-scope fences); 8 teams by XCD, of
            # which 6 stay empty
            for tc, slots in ((2, 0), (1, 3), (8, 0)):
                tctx = sbc.Context(0, {"team_wg_waves": 4, "slots": slots, "batch_wg_waves": 4, "team_count": tc,
                                       "team_min_vertices": 3})
                sizes = (5, 65, 130) if tc == 2 or full else (65,)
                for n in sizes:
                    r = gg.rng(n * 11 + tc)
                    g = gg.erdos_renyi(n, min(0.9, 6.0 / max(n - 1, 1)), int(r.integers(1 << 30)))
                    reach, ident = gg.random_attributes(n, int(r.integers(1 << 30)), rmax=5, kmax=3)
                    for rr, kk in ((None, None), (reach, ident)):
                        want = oracle.bc_weighted(g.n, g.row_ptr, g.col, rr, kk)
                        got = sbc.sbc_piece_bc(tctx.h, g.n, g.row_ptr, g.col, rr, kk, kernel=4)
                        assert_bc_close(got, want, 1e-9, f"team piece n={n} teams={tc}")
                if tc == 2 or full:
                    for name, g in (("rmat6", gg.rmat_decorated(scale=6, seed=3)),
                                    ("decorated", gg.decorated_random(30, 0.1, 8, 5, 3, 11))):
                        want = oracle.bc(g)
                        for mode in ("plain", "compressed"):
                            got = sbc.betweenness(g.n, g.row_ptr, g.col, mode=mode, ctx=tctx)
                            assert_bc_close(got, want, 1e-9, f"team {name}/{mode} teams={tc}")
                        got = sbc.betweenness(g.n, g.row_ptr, g.col, mode="compressed", ops="odasi", ctx=tctx)
                        assert_bc_close(got, want, 1e-9, f"team {name}/odasi teams={tc}")
                print(f"   teams={tc} slots={slots} ok", flush=True)
                tctx.close()
        check("team kernel", team)

        def team_hubs():
            n = 1300
            r = gg.rng(5)
            u = np.concatenate([np.zeros(1200, np.int64), r.integers(1, n, 600)])
            v = np.concatenate([np.arange(1, 1201), r.integers(1, n, 600)])
            g2 = gg.csr_from_edges(n, u, v)
            src = np.arange(0, 16, dtype=np.int32)
            want = oracle.bc_plain(g2.n, g2.row_ptr, g2.col, sources=src)
            tctx = sbc.Context(0, {"team_wg_waves": 4, "slots": 0, "batch_wg_waves": 4, "team_count": 2, "team_min_vertices": 64,
                                   "team_split_arcs": 512})
            G = sbc.Graph(g2.n, g2.row_ptr, g2.col)
            got = sbc.sbc_betweenness_sources(tctx.h, G.h, src)
            assert_bc_close(got, want, 1e-9, "team hub rows")
            tctx.close()
            # a low split threshold: many rows of every level are pulled in slices
            tctx = sbc.Context(0, {"team_wg_waves": 4, "slots": 0, "batch_wg_waves": 4, "team_count": 2, "team_min_vertices": 3,
                                   "team_split_arcs": 64})
            for g in (gg.rmat_decorated(scale=7, seed=5), gg.complete_bipartite(40, 80)):
                want = oracle.bc(g)
                for mode in ("plain", "compressed"):
                    got = sbc.betweenness(g.n, g.row_ptr, g.col, mode=mode, ctx=tctx)
                    assert_bc_close(got, want, 1e-9, f"team split 64 n={g.n}/{mode}")
            tctx.close()
        check("team split rows", team_hubs)

        def team_phases():
            g = gg.rmat_decorated(scale=7, seed=3)
            pctx = sbc.Context(0, {"team_wg_waves": 4, "slots": 0, "batch_wg_waves": 4, "team_count": 2, "team_min_vertices": 3,
                                   "profile_phases": 1})
            G = sbc.Graph(g.n, g.row_ptr, g.col)
            G.preprocess("dai")
            plan = sbc.sbc_plan_create(pctx.h, G.h, sbc.SBC_COMPRESSED)
            sbc.sbc_plan_execute(plan)
            st = sbc.sbc_plan_sync(plan)
            ph = sbc.sbc_plan_phase_profile(plan)
            assert_bc_close(sbc.sbc_plan_result(plan, g.n), oracle.bc(g), 1e-9, "profiled team run")
            sbc.sbc_plan_destroy(plan)
            assert st["items_class"][4] >= 1 and st["grid_class"][4] == 4, st
            assert ph["items"] >= 1 and ph["entries"] >= ph["items"] and ph["team_sync_ms"] >= 0, ph
            print("   phases", {k: round(v, 3) for k, v in ph.items()}, flush=True)
            pctx.close()
        check("team phase timers", team_phases)

        def team_abort():
            # no barrier waiting allowed: the team aborts, every wave leaves the
            # kernel, and the run reports a device error instead of hanging
            g = gg.rmat_decorated(scale=6, seed=3)
            actx = sbc.Context(0, {"team_wg_waves": 4, "slots": 0, "batch_wg_waves": 4, "team_count": 1, "team_min_vertices": 3,
                                   "team_spin_ms": 0})
            try:
                sbc.betweenness(g.n, g.row_ptr, g.col, mode="compressed", ctx=actx)
            except sbc.SbcError as e:
                assert e.status == -8 and "team barrier" in str(e), e
            else:
                raise AssertionError("aborted team run reported success")
            actx.close()
        check("team abort path", team_abort)
    if "wave" in which:
        def wave():
            # the small-piece kernel: forced on single pieces (few and many
            # levels, a hub, items of a few sources), and by default routing
            # on graphs that shatter into small pieces
            wctx = sbc.Context(0, {"team_wg_waves": 4, "slots": 2, "batch_wg_waves": 4, "deep_wg_waves": 4})
            cases = [("er3", gg.erdos_renyi(3, 0.9, 1)), ("er5", gg.erdos_renyi(5, 0.9, 2)),
                     ("er65", gg.erdos_renyi(65, 0.1, 3)), ("er130", gg.erdos_renyi(130, 0.05, 4)),
                     ("cycle40", gg.cycle(40)), ("K9", gg.complete(9)), ("K3,70", gg.complete_bipartite(3, 70))]
            if full:
                cases += [("er256", gg.erdos_renyi(256, 0.03, 5)), ("path200", gg.path(200))]
            for name, g in cases:
                r = gg.rng(g.n)
                reach, ident = gg.random_attributes(g.n, int(r.integers(1 << 30)), rmax=5, kmax=3)
                for rr, kk in ((None, None), (reach, ident)):
                    want = oracle.bc_weighted(g.n, g.row_ptr, g.col, rr, kk)
                    got = sbc.sbc_piece_bc(wctx.h, g.n, g.row_ptr, g.col, rr, kk, kernel=5)
                    assert_bc_close(got, want, 1e-9, f"wave piece {name}")
                print(f"   {name} n={g.n} ok", flush=True)
            sbc.sbc_context_set_param(wctx.h, "wave_sources_per_item", 7)
            g = gg.erdos_renyi(40, 0.15, 8)
            want = oracle.bc_weighted(g.n, g.row_ptr, g.col, None, None)
            assert_bc_close(sbc.sbc_piece_bc(wctx.h, g.n, g.row_ptr, g.col, None, None, kernel=5), want, 1e-9,
                            "wave piece, 7-source items")
            sbc.sbc_context_set_param(wctx.h, "wave_sources_per_item", 64)
            big = gg.erdos_renyi(2100, 0.003, 9)
            try:
                sbc.sbc_piece_bc(wctx.h, big.n, big.row_ptr, big.col, None, None, kernel=5)
            except sbc.SbcError as e:
                assert e.status == -1, e
            else:
                raise AssertionError("a piece beyond the small-piece LDS was accepted")
            for name, g in (("blocks", gg.block_tree(n_pieces=12, max_size=90, seed=13)),
                            ("rmat7", gg.rmat_decorated(scale=7, seed=3))):
                want = oracle.bc(g)
                for mode in ("plain", "compressed"):
                    G = sbc.Graph(g.n, g.row_ptr, g.col)
                    if mode == "compressed":
                        G.preprocess("odai")
                    plan = sbc.sbc_plan_create(wctx.h, G.h, sbc._mode(mode))
                    sbc.sbc_plan_execute(plan)
                    st = sbc.sbc_plan_sync(plan)
                    assert_bc_close(sbc.sbc_plan_result(plan, g.n), want, 1e-9, f"wave routing {name}/{mode}")
                    sbc.sbc_plan_destroy(plan)
                    assert mode == "plain" and g.n > 256 or st["items_class"][0] >= 1, st
                print(f"   routed {name} ok", flush=True)
            wctx.close()
        check("small-piece kernel", wave)
    if "noalloc" in which:
        def noalloc():
            # the entry point without device allocation: "device" buffers are
            # host memory in the emulation; two calls in a row, the second
            # smaller, each equal to sbc_piece_bc; then a refused size
            for n, seed in ((300, 21), (70, 22)):
                r = gg.rng(seed)
                g = gg.erdos_renyi(n, 6.0 / n, seed)
                reach, ident = gg.random_attributes(n, int(r.integers(1 << 30)), rmax=4, kmax=3)
                want = sbc.sbc_piece_bc(ctx.h, g.n, g.row_ptr, g.col, reach, ident, kernel=3)
                rp, cl = np.ascontiguousarray(g.row_ptr, np.int32), np.ascontiguousarray(g.col, np.int32)
                rc, kc = np.ascontiguousarray(reach, np.int32), np.ascontiguousarray(ident, np.int32)
                out = np.full(n, 7.0)
                flags = np.full(1, -1, np.int32)
                sbc.sbc_piece_bc_noalloc(ctx.h, n, len(cl), rp.ctypes.data, cl.ctypes.data, rc.ctypes.data,
                                         kc.ctypes.data, out.ctypes.data, flags.ctypes.data)
                assert flags[0] == 0, flags
                assert_bc_close(out, want, 1e-9, f"noalloc n={n}")
                print(f"   n={n} ok", flush=True)
            try:
                sbc.sbc_piece_bc_noalloc(ctx.h, 65537, 0, rp.ctypes.data, cl.ctypes.data, None, None,
                                         out.ctypes.data)
            except sbc.SbcError as e:
                assert e.status == -6, e
            else:
                raise AssertionError("an oversized piece was accepted")
        check("no-allocation entry point", noalloc)
    if "server" in which:
        def server():
            gs = [gg.rmat_decorated(scale=7, seed=s) for s in range(3)] + [gg.grid_deleted(side=10, seed=4)]
            srv = sbc.sbc_server_create(ctx.h, 2, 0)
            Gs = [sbc.Graph(g.n, g.row_ptr, g.col) for g in gs]
            jobs = [sbc.sbc_server_submit(srv, G.h, sbc.SBC_COMPRESSED) for G in Gs]
            for g, j in zip(gs, jobs):
                got, st = sbc.sbc_job_wait(j, g.n)
                assert_bc_close(got, oracle.bc(g), 1e-9, "server job")
                sbc.sbc_job_release(j)
            sbc.sbc_server_destroy(srv)
        check("server", server)
    if "far" in which:
        def far():
            # farness kernel: per-piece sums equal to the oracle's exactly, and
            # the whole farness after the host pass; two slots reused by many
            # items, levels wider than a workgroup, weighted and unweighted pieces
            fctx = sbc.Context(0, {"team_wg_waves": 4, "far_wg_waves": 4, "slots": 2})
            cases = [("decorated", gg.decorated_random(60, 0.06, 15, 4, 4, 5)), ("grid", gg.grid2d(9, 11)),
                     ("blocks", gg.block_tree(n_pieces=10, max_size=80, seed=2)), ("er400", gg.erdos_renyi(400, 0.02, 6)),
                     ("path3", gg.path(3)), ("K5", gg.complete(5))]
            for name, g in cases:
                want = oracle.farness(g.n, g.row_ptr, g.col)
                for ops in ("oda", ""):
                    G = sbc.Graph(g.n, g.row_ptr, g.col)
                    f, _ = sbc.sbc_far_create(G.h, ops)
                    ex = sbc.sbc_far_export(f)
                    far, clo, st, W = sbc.sbc_far_run(fctx.h, f, g.n, with_piece_sums=True)
                    if len(ex["vtx_off"]) > 1:
                        wantW = oracle.farness_pieces(ex["vtx_off"], ex["row"], ex["col"], ex["reach"])
                        assert np.array_equal(W, wantW), (name, ops)
                    assert np.array_equal(far, want), (name, ops)
                    assert st["flags"] == 0, st
                    sbc.sbc_far_destroy(f)
                    G.close()
                print(f"   {name} ok", flush=True)
            fctx.close()
        check("farness kernel", far)
    print("ALL OK", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["single", "pieces", "whole", "hubs", "team", "wave", "noalloc", "server", "far"])
