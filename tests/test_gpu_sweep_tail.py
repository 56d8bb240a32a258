"""The filter sweeps after the schedule's separate launches run in one launch
whose blocks wait for each other between sweeps.  Sums are integers and
every point's arithmetic is the same, so any split of the sweeps between the
two gives the same bits: checked for one cloud and for a batch whose clouds
stop at different q, for the filter on a stored graph, for the generic K path
(where the looping grid may not fit on the device and the sweeps fall back to
separate launches), and for a captured graph."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2401_09721_amd import fgbd, synth  # noqa: E402

from gpu_helpers import compare_denoise, dev  # noqa: E402

pytestmark = pytest.mark.gpu


def cloud(seed, target, sigma):
    c = synth.random_shapes_cloud(seed, bits=8, n_ellipsoids=3, target=target, sigma=sigma)
    return c.xyz, c.noisy


def denoise_with(ctx, xyz, rgb, prm, launches, sweep_blocks=1024):
    ctx.set_schedule(1024, 1024, sweep_blocks, launches)
    out, res = fgbd.denoise(dev(xyz, torch.int32), dev(rgb, torch.float32), prm, ctx=ctx)
    torch.cuda.synchronize()
    return out.cpu().numpy(), fgbd.read_result(res)


def test_single_cloud_every_split_same_bits():
    prm = fgbd.default_params(bits=8)
    xyz, rgb = cloud(81, 20000, 35.0)
    ctx = fgbd.Context("cuda")
    ref, rr = denoise_with(ctx, xyz, rgb, prm, 1024)
    assert rr["sweeps"] >= 4, rr  # enough sweeps for the splits below to reach the in-launch loop
    for launches in (1, 2, 3, rr["sweeps"], rr["sweeps"] + 1):
        out, r = denoise_with(ctx, xyz, rgb, prm, launches)
        assert np.array_equal(out, ref), launches
        assert r == rr, launches
    out, r = denoise_with(ctx, xyz, rgb, prm, 1)
    compare_denoise(out, r, xyz, rgb, prm)
    ctx.close()


def test_batch_clouds_stop_at_different_q():
    prm = fgbd.default_params(bits=8)
    clouds = [cloud(91, 12000, 35.0), cloud(92, 3000, 5.0), cloud(93, 8000, 20.0), cloud(94, 500, 30.0)]
    xyz = np.concatenate([c[0] for c in clouds])
    rgb = np.concatenate([c[1] for c in clouds])
    offs = np.concatenate([[0], np.cumsum([len(c[0]) for c in clouds])]).astype(np.int64)
    ctx = fgbd.Context("cuda")

    def run(launches):
        ctx.set_schedule(1024, 1024, 1024, launches)
        out, res = fgbd.denoise_batched(dev(xyz, torch.int32), dev(rgb, torch.float32), dev(offs, torch.int64), prm,
                                        ctx=ctx)
        torch.cuda.synchronize()
        return out.cpu().numpy(), fgbd.read_results(res)

    ref, rr = run(1024)
    assert len({r["sweeps"] for r in rr}) > 1, rr  # the clouds really stop at different sweeps
    for launches in (1, 2, 4):
        out, r = run(launches)
        assert np.array_equal(out, ref), launches
        assert r == rr, launches
    ctx.close()


@pytest.mark.parametrize("k", [8, 6])
def test_filter_on_stored_graph_split(k):
    """fgbd_filter on a stored graph (weights read from p): the selected
    filter under every split, and fixed q (always one launch per sweep)."""
    prm = fgbd.default_params(bits=8, k=k)
    xyz, rgb = cloud(101, 15000, 35.0)
    ctx = fgbd.Context("cuda")
    g = fgbd.build_slg(dev(xyz, torch.int32), prm, ctx=ctx)
    x = dev(rgb, torch.float32)
    noise, spread, _ = fgbd.estimate_noise(g, x, prm, ctx=ctx)
    sel, fixed = [], []
    for launches in (1024, 1, 3):
        ctx.set_schedule(1024, 1024, 1024, launches)
        out, res = fgbd.filter(g, x, prm, noise=noise, spread=spread, ctx=ctx)
        torch.cuda.synchronize()
        sel.append((out.cpu().numpy(), fgbd.read_result(res)))
        out, res = fgbd.filter(g, x, prm, q_fixed=7, ctx=ctx)
        torch.cuda.synchronize()
        r = fgbd.read_result(res)
        assert r["q"] == 7 and r["sweeps"] == 7
        fixed.append(out.cpu().numpy())
    assert sel[0][1]["sweeps"] >= 4, sel[0][1]
    for out, r in sel[1:]:
        assert np.array_equal(out, sel[0][0]) and r == sel[0][1]
    assert np.array_equal(fixed[0], fixed[1]) and np.array_equal(fixed[0], fixed[2])
    ctx.close()


@pytest.mark.parametrize("sweep_blocks", [1024, 256])
def test_generic_k_split(sweep_blocks):
    """K = 6 (the generic kernel, more registers): with 1024 sweep blocks the
    looping grid may not fit and every sweep is a launch of its own; with 256
    it fits.  Same bits either way."""
    prm = fgbd.default_params(bits=8, k=6)
    xyz, rgb = cloud(111, 12000, 35.0)
    ctx = fgbd.Context("cuda")
    ref, rr = denoise_with(ctx, xyz, rgb, prm, 1024, sweep_blocks)
    out, r = denoise_with(ctx, xyz, rgb, prm, 1, sweep_blocks)
    assert np.array_equal(out, ref) and r == rr
    compare_denoise(out, r, xyz, rgb, prm)
    ctx.close()


def test_captured_graph_with_looped_sweeps():
    """One capture with 2 separate sweep launches, replayed on frames that need
    more sweeps than that: every replay equals the eager call."""
    prm = fgbd.default_params(bits=8)
    cap = 20000
    ctx = fgbd.Context("cuda")
    ctx.reserve(prm, cap, 1)
    ctx.set_schedule(1024, 1024, 1024, 2)
    xyz_s = torch.zeros((cap, 3), dtype=torch.int32, device="cuda")
    rgb_s = torch.zeros((cap, 3), dtype=torch.float32, device="cuda")
    off_s = torch.zeros(2, dtype=torch.int64, device="cuda")
    out_s = torch.zeros((cap, 3), dtype=torch.float32, device="cuda")
    res_s = fgbd.new_result("cuda", 1)

    def load(xyz, rgb):
        n = len(xyz)
        xyz_s.zero_()
        rgb_s.zero_()
        xyz_s[:n] = dev(xyz, torch.int32)
        rgb_s[:n] = dev(rgb, torch.float32)
        off_s.copy_(torch.tensor([0, n], dtype=torch.int64))

    frames = [cloud(121 + f, t, s) for f, (t, s) in enumerate([(16000, 35.0), (9000, 20.0), (19000, 30.0)])]
    frames = [f for f in frames if len(f[0]) <= cap]
    assert len(frames) >= 2
    load(*frames[0])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside the capture
        fgbd.denoise_batched(xyz_s, rgb_s, off_s, prm, ctx=ctx, out=out_s, res=res_s)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fgbd.denoise_batched(xyz_s, rgb_s, off_s, prm, ctx=ctx, out=out_s, res=res_s)
    torch.cuda.synchronize()
    saw_tail = False
    for f, (xyz, rgb) in enumerate(frames + frames[:1]):
        load(xyz, rgb)
        out_s.fill_(-7.0)
        graph.replay()
        torch.cuda.synchronize()
        got = out_s.cpu().numpy().copy()
        got_r = fgbd.read_results(res_s)[0]
        saw_tail |= got_r["sweeps"] > 2
        ref_out = torch.full((cap, 3), -7.0, dtype=torch.float32, device="cuda")
        ref_res = fgbd.new_result("cuda", 1)
        fgbd.denoise_batched(xyz_s, rgb_s, off_s, prm, ctx=ctx, out=ref_out, res=ref_res)
        torch.cuda.synchronize()
        assert np.array_equal(got, ref_out.cpu().numpy()), f"frame {f}: replay differs from eager"
        assert got_r == fgbd.read_results(ref_res)[0]
    assert saw_tail
    ctx.close()


def test_adaptive_launch_count_keeps_bits():
    """Eager calls lower their separate sweep launches to what recent calls
    needed (read back without waiting); a frame that needs more sweeps than
    that runs the rest in the looping launch.  A stream of frames whose
    sweep counts jump up and down gives, frame by frame, the bits of a fresh
    context (no history) on the same frame."""
    prm = fgbd.default_params(bits=8)
    frames = [cloud(131, 15000, 5.0), cloud(132, 15000, 5.0), cloud(133, 15000, 35.0), cloud(134, 15000, 20.0),
              cloud(135, 15000, 5.0), cloud(136, 15000, 35.0)]
    ctx = fgbd.Context("cuda")
    seen = set()
    for rep in range(3):
        for f, (xyz, rgb) in enumerate(frames):
            out, res = fgbd.denoise(dev(xyz, torch.int32), dev(rgb, torch.float32), prm, ctx=ctx)
            torch.cuda.synchronize()  # lets the next call read this call's sweep count
            r = fgbd.read_result(res)
            fresh = fgbd.Context("cuda")
            ref, rres = fgbd.denoise(dev(xyz, torch.int32), dev(rgb, torch.float32), prm, ctx=fresh)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref.cpu().numpy()), (rep, f)
            assert r == fgbd.read_result(rres), (rep, f)
            fresh.close()
            seen.add(r["sweeps"])
    assert max(seen) - min(seen) >= 2, seen  # the counts really vary
    ctx.close()


def test_wait_bound_zero_gives_up_with_defined_output():
    """The in-launch sweep loop's wait bound set to 0 from the host: the loop
    gives up at its first wait that is not already over, every block still
    exits normally, the result carries FGBD_ST_SWEEP_STALL, the binding raises
    on reading it, and every output row holds either the input colour or the
    colour the unstalled call produces (no row is left unwritten).  The default
    bound then gives the normal result again on the same context."""
    prm = fgbd.default_params(bits=8)
    xyz, rgb = cloud(81, 20000, 35.0)
    ctx = fgbd.Context("cuda")
    ref, rr = denoise_with(ctx, xyz, rgb, prm, 1024)  # every sweep a launch of its own: no waits
    assert rr["sweeps"] >= 3, rr
    ctx.set_sweep_wait(0)
    ctx.set_schedule(1024, 1024, 1024, 1)
    out = torch.full((len(xyz), 3), float("nan"), device="cuda")
    out, res = fgbd.denoise(dev(xyz, torch.int32), dev(rgb, torch.float32), prm, ctx=ctx, out=out)
    torch.cuda.synchronize()
    with pytest.raises(fgbd.FgbdStallError):
        fgbd.read_result(res)
    r = fgbd.read_result(res, check=False)
    assert r["status"] & fgbd.FGBD_ST_SWEEP_STALL
    o = out.cpu().numpy()
    as_input = np.all(o == rgb, axis=1)
    as_filtered = np.all(o == ref, axis=1)
    assert np.all(as_input | as_filtered)
    assert as_input.sum() > 0
    ctx.set_sweep_wait(-1)
    out2, r2 = denoise_with(ctx, xyz, rgb, prm, 1)
    assert np.array_equal(out2, ref) and r2 == rr
    ctx.close()


def test_steady_sweep_counts_finalise_in_the_tail():
    """Calls whose recent sweep counts agree launch exactly as many separate
    sweeps as the selection needed lately, and the finalising launch applies
    the last sweep's sums itself before it finalises.  The same frame (and
    the same batch) called again and again on one context gives, every time,
    the bits of a fresh context."""
    prm = fgbd.default_params(bits=8)
    xyz, rgb = cloud(141, 15000, 20.0)
    fresh = fgbd.Context("cuda")
    ref, rres = fgbd.denoise(dev(xyz, torch.int32), dev(rgb, torch.float32), prm, ctx=fresh)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    rres = fgbd.read_result(rres)
    fresh.close()
    ctx = fgbd.Context("cuda")
    for rep in range(6):
        out, res = fgbd.denoise(dev(xyz, torch.int32), dev(rgb, torch.float32), prm, ctx=ctx)
        torch.cuda.synchronize()  # lets the next call read this call's sweep count
        assert np.array_equal(out.cpu().numpy(), ref), rep
        assert fgbd.read_result(res) == rres, rep
    # a batch of three clouds with different noise levels, called repeatedly
    parts = [cloud(142, 9000, 5.0), cloud(143, 12000, 20.0), cloud(144, 7000, 35.0)]
    bx = dev(np.concatenate([p[0] for p in parts]), torch.int32)
    bc = dev(np.concatenate([p[1] for p in parts]), torch.float32)
    offs = torch.tensor(np.concatenate([[0], np.cumsum([len(p[0]) for p in parts])]), dtype=torch.int64,
                        device="cuda")
    fresh = fgbd.Context("cuda")
    bref, bres = fgbd.denoise_batched(bx, bc, offs, prm, ctx=fresh)
    torch.cuda.synchronize()
    bref = bref.cpu().numpy()
    bres = fgbd.read_results(bres)
    fresh.close()
    for rep in range(6):
        out, res = fgbd.denoise_batched(bx, bc, offs, prm, ctx=ctx)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), bref), rep
        assert fgbd.read_results(res) == bres, rep
    ctx.close()
