"""The batched step with problem descriptors in device memory
(nmf_beta_step_batched): planned on the device by one workgroup, run by the
persistent kernel of nmf_batch_step.

Its results must equal, bit for bit, those of the host-planned batch
(nmf_batch_create + nmf_batch_step) on the same problems with the same tile
table: both run the same kernels on the same splits, so only the workspace
addresses differ.  One step is also held to the oracle gates (tests/gates.py).
The call is captured into a graph and replayed after the descriptors change
(other matrices, shapes, betas, fewer problems through the device count), each
replay checked against an eager host-planned batch.  Invalid descriptors,
overlaps and plans beyond the reserved capacity leave everything untouched and
set NMF_FLAG_SKIPPED.  The tuner of the per-bucket tile table writes and reads
its cache file.
"""
import os

import numpy as np
import pytest
import torch

import oracle as O
import synth
import paper_2106_15214_amd as nb
from gates import check_pair

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
E_WS, E_UNSUP = 5, 7

SPECS = [(64, 100, 5, 1.0), (200, 150, 20, 0.0), (257, 300, 49, 0.5), (130, 70, 64, 2.0), (33, 1000, 8, 1.5),
         (1, 40, 3, 1.2), (40, 1, 3, 2.5), (129, 129, 1, -0.5), (96, 160, 32, 1.0), (300, 97, 33, 0.0),
         (500, 260, 17, 2.0), (77, 611, 60, 0.5), (1100, 2100, 40, 1.0), (700, 4500, 12, 0.5)]
WELL_POSED = [s for s in SPECS if s[2] < min(s[0], s[1])]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def make_set(specs, seed0):
    out = []
    for i, (F, N, K, beta) in enumerate(specs):
        p = synth.random_positive(F, N, K, seed=seed0 + i, zeros=0.1 if beta > 0 else 0.0)
        out.append((p.V, p.W, p.H, beta))
    return out


def to_dev(probs):
    return [(dev(V), dev(W), dev(H), b) for V, W, H, b in probs]


def reserve_for(ctx, shapes, mode, slots=None, precision="fp32"):
    items, nbytes = nb.batch_requirements(shapes, mode, nb.get_batch_tiles(ctx), precision)
    nb.reserve_batched(slots or len(shapes), items, nbytes, ctx=ctx)
    return items, nbytes


def shapes_of(probs):
    return [(V.shape[0], V.shape[1], W.shape[1], beta) for V, W, H, beta in probs]


def bits(t):
    return t.view(torch.int64 if t.dtype == torch.float64 else torch.int32)


def assert_same(a, b, what):
    """Bitwise equality of every W and H (NaN patterns included)."""
    for i, ((_, Wa, Ha, _), (_, Wb, Hb, _)) in enumerate(zip(a, b)):
        assert torch.equal(bits(Wa), bits(Wb)) and torch.equal(bits(Ha), bits(Hb)), f"{what}: problem {i}"


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("mode", ["joint", "alternating"])
def test_device_planned_equals_host_planned(mode, precision):
    probs = make_set(SPECS, seed0=2000)
    a, b = to_dev(probs), to_dev(probs)
    print(f"[device batch] {mode} {precision} problems={len(a)}", flush=True)
    ctx = nb.Context(0)
    ctx.set_path("stream")
    reserve_for(ctx, shapes_of(probs), mode, precision=precision)
    dp = nb.DeviceProblems(len(a))
    dp.set(a)
    host = nb.Batch(b, mode, precision=precision, ctx=ctx)
    oa = torch.zeros(len(a), dtype=torch.float64, device=DEV)
    ob = torch.zeros(len(a), dtype=torch.float64, device=DEV)
    for t in range(3):
        nb.step_batched(dp, mode, precision=precision, objectives=oa, ctx=ctx)
        host.step(objectives=ob)
        torch.cuda.synchronize()
        assert torch.equal(bits(oa), bits(ob)), t
        assert_same(a, b, f"step {t}")
    # the ill-posed problems (K >= min(F, N)) may reach 0/0 in later steps:
    # both paths report the same flags
    hf, df = host.flags(), nb.get_flags(clear=True, ctx=ctx)
    assert hf == df and df & ~nb.FLAG_NONFINITE == 0, (hf, df)
    host.close()
    ctx.close()


@pytest.mark.parametrize("mode", ["joint", "alternating"])
def test_device_planned_step_matches_oracle(mode):
    probs = make_set(SPECS, seed0=2100)
    d = to_dev(probs)
    ctx = nb.Context(0)
    reserve_for(ctx, shapes_of(probs), mode)
    dp = nb.DeviceProblems(len(d))
    dp.set(d)
    obj = torch.full((len(d),), float("nan"), dtype=torch.float64, device=DEV)
    print(f"[device batch] oracle {mode}", flush=True)
    nb.step_batched(dp, mode, objectives=obj, ctx=ctx)
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx) == 0
    o = obj.cpu().numpy()
    f = O.jmm_iteration if mode == "joint" else O.bmm_iteration
    for i, ((V, W, H, beta), (_, Wd, Hd, _)) in enumerate(zip(probs, d)):
        V64, W64, H64 = V.astype(np.float64), W.astype(np.float64), H.astype(np.float64)
        Wr, Hr = f(V64, W64, H64, beta)
        check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr, tag=f"device-planned problem {i} beta={beta}")
        d0 = O.objective(V64, W64, H64, beta)
        assert abs(o[i] - d0) <= 1e-6 * abs(d0), (i, o[i], d0)
    ctx.close()


def test_graph_replay_over_changing_descriptors():
    """One capture, replayed over three descriptor sets of other shapes and
    betas (the last one with fewer problems through the device count)."""
    mode = "joint"
    sets = [make_set(WELL_POSED, seed0=2200),
            make_set([(s[1] % 700 + 20, s[0] + 50, max(1, s[2] // 2), 2.0 - s[3] / 2) for s in WELL_POSED], 2300),
            make_set(WELL_POSED[:5], seed0=2400)]
    ctx = nb.Context(0)
    slots = max(len(s) for s in sets)
    need_items, need_bytes = 0, 0
    for s in sets:
        i, b = nb.batch_requirements(shapes_of(s), mode, nb.get_batch_tiles(ctx))
        need_items, need_bytes = max(need_items, i), max(need_bytes, b)
    nb.reserve_batched(slots, need_items, need_bytes, ctx=ctx)
    dp = nb.DeviceProblems(slots)
    dcount = torch.tensor([slots], dtype=torch.int32, device=DEV)
    obj = torch.zeros(slots, dtype=torch.float64, device=DEV)
    first = to_dev(sets[0])
    dp.set(first)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    print("[device batch] capture", flush=True)
    with torch.cuda.graph(g, stream=s):
        nb.step_batched(dp, mode, count=slots, objectives=obj, d_count=dcount, stream=s, ctx=ctx)
    # capture launches nothing: the first set is still untouched
    torch.cuda.synchronize()
    assert_same(first, to_dev(sets[0]), "after capture")
    for rep, probs in enumerate(sets + [sets[0]]):
        print(f"[device batch] replay {rep} problems={len(probs)}", flush=True)
        d = to_dev(probs)
        ref = to_dev(probs)
        dp.set(d)
        dcount.fill_(len(d))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        host = nb.Batch(ref, mode, ctx=ctx)
        oref = torch.zeros(len(ref), dtype=torch.float64, device=DEV)
        host.step(objectives=oref)
        torch.cuda.synchronize()
        assert_same(d, ref, f"replay {rep}")
        assert torch.equal(bits(obj[:len(d)]), bits(oref)), rep
        assert host.flags() == 0
        host.close()
        assert nb.get_flags(clear=True, ctx=ctx) == 0, rep
        # eager work between the replays
        r = synth.random_positive(90, 120, 7, seed=2500 + rep)
        nb.step(dev(r.V), dev(r.W), dev(r.H), 2.0, "alternating", ctx=ctx)
        torch.cuda.synchronize()
    # re-reserving is refused once a batched call was captured
    with pytest.raises(nb.NmfError) as e:
        nb.reserve_batched(slots, need_items, need_bytes, ctx=ctx)
    assert e.value.status == E_WS
    del g
    ctx.close()


def test_skipped_batches_leave_everything_untouched():
    mode = "joint"
    probs = to_dev(make_set(WELL_POSED, seed0=2600))
    keep = [(W.clone(), H.clone()) for _, W, H, _ in probs]
    ctx = nb.Context(0)
    items, nbytes = reserve_for(ctx, shapes_of(probs), mode)
    dp = nb.DeviceProblems(len(probs))
    obj = torch.full((len(probs),), -7.0, dtype=torch.float64, device=DEV)

    def run_and_check(tag, count=None, d_count=None):
        print(f"[device batch] skip case: {tag}", flush=True)
        nb.step_batched(dp, mode, count=count, objectives=obj, d_count=d_count, ctx=ctx)
        torch.cuda.synchronize()
        assert nb.get_flags(clear=True, ctx=ctx) == nb.FLAG_SKIPPED, tag
        for i, ((_, W, H, _), (W0, H0)) in enumerate(zip(probs, keep)):
            assert torch.equal(W, W0) and torch.equal(H, H0), (tag, i)
        assert torch.all(obj == -7.0), tag

    # an invalid descriptor (K = 0) among valid ones
    raw = bytearray(nb.DeviceProblems.pack(probs))
    bad = bytearray(raw)
    sz = len(raw) // len(probs)
    bad[2 * sz + 16:2 * sz + 24] = (0).to_bytes(8, "little")  # problem 2: K = 0
    dp.set_raw(bytes(bad))
    dp.count = len(probs)
    run_and_check("K = 0")
    # non-finite beta
    bad = bytearray(raw)
    bad[3 * sz + sz - 8:3 * sz + sz] = np.float64(np.nan).tobytes()
    dp.set_raw(bytes(bad))
    run_and_check("beta = nan")
    # problem 1 updates problem 0's W (descriptor fields: F N K V ldv W ldw H ldh beta)
    assert sz == 80
    bad = bytearray(raw)
    bad[sz + 40:sz + 48] = probs[0][1].data_ptr().to_bytes(8, "little")
    dp.set_raw(bytes(bad))
    run_and_check("W shared between problems")
    # problem 0's W inside problem 1's V
    bad = bytearray(raw)
    bad[sz + 24:sz + 32] = probs[0][1].data_ptr().to_bytes(8, "little")  # problem 1: V = problem 0's W
    dp.set_raw(bytes(bad))
    run_and_check("W inside another problem's V")
    # a device count outside 0..count
    dp.set(probs)
    dcount = torch.tensor([len(probs) + 1], dtype=torch.int32, device=DEV)
    run_and_check("device count too large", d_count=dcount)
    dcount.fill_(-1)
    run_and_check("negative device count", d_count=dcount)
    # more workspace than reserved: a region one byte short
    nb.reserve_batched(len(probs), items, nbytes - 1, ctx=ctx)
    run_and_check("workspace over capacity")
    nb.reserve_batched(len(probs), items - 1, nbytes, ctx=ctx)
    run_and_check("queue over capacity")
    # exactly the requirements: runs
    nb.reserve_batched(len(probs), items, nbytes, ctx=ctx)
    dcount.fill_(0)
    nb.step_batched(dp, mode, objectives=obj, d_count=dcount, ctx=ctx)  # zero problems: nothing, no flag
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx) == 0
    assert torch.all(obj == -7.0)
    nb.step_batched(dp, mode, objectives=obj, ctx=ctx)
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx) == 0
    assert not torch.any(obj == -7.0)
    ctx.close()


def test_host_side_status_codes():
    probs = to_dev(make_set(WELL_POSED[:3], seed0=2700))
    ctx = nb.Context(0)
    dp = nb.DeviceProblems(3)
    dp.set(probs)
    with pytest.raises(nb.NmfError) as e:  # nothing reserved
        nb.step_batched(dp, "joint", ctx=ctx)
    assert e.value.status == E_WS
    reserve_for(ctx, shapes_of(probs), "joint", slots=2)
    with pytest.raises(nb.NmfError) as e:  # more descriptors than slots
        nb.step_batched(dp, "joint", ctx=ctx)
    assert e.value.status == E_WS
    with pytest.raises(nb.NmfError) as e:
        nb.step_batched(dp, "joint", count=2, precision="fp16", ctx=ctx)
    assert e.value.status == E_UNSUP
    nb.step_batched(dp, "joint", count=2, ctx=ctx)
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx) == 0
    ctx.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_tile_table_changes_plans_not_results(precision):
    """A table with other tiles per item splits the contractions differently:
    the device-planned step then equals the host batch built with that table
    and stays within the oracle gates."""
    probs = make_set([(1100, 2100, 40, 1.0), (700, 4500, 12, 0.5), (300, 97, 33, 0.0)], seed0=2800)
    a, b = to_dev(probs), to_dev(probs)
    print(f"[device batch] custom table {precision}", flush=True)
    ctx = nb.Context(0)
    tiles = [(4, 8, 16, 32, 64, 128)[b % 6] for b in range(nb.BATCH_BUCKETS)]
    nb.set_batch_tiles(tiles, ctx=ctx)
    assert nb.get_batch_tiles(ctx) == tiles
    reserve_for(ctx, shapes_of(probs), "joint", precision=precision)
    dp = nb.DeviceProblems(len(a))
    dp.set(a)
    nb.step_batched(dp, "joint", precision=precision, ctx=ctx)
    host = nb.Batch(b, "joint", precision=precision, ctx=ctx)  # tiles_per_item 0: the context's table
    host.step()
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx) == 0 and host.flags() == 0
    assert_same(a, b, "custom table")
    host.close()
    for (V, W, H, beta), (_, Wd, Hd, _) in zip(probs, a):
        Wr, Hr = O.jmm_iteration(V.astype(np.float64), W.astype(np.float64), H.astype(np.float64), beta)
        check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr, precision, beta,
                   tag=f"custom table {precision}, beta={beta}")
    if precision == "bf16":
        ctx.close()
        return
    with pytest.raises(nb.NmfError):
        nb.set_batch_tiles([0] * nb.BATCH_BUCKETS, ctx=ctx)
    with pytest.raises(ValueError):
        nb.set_batch_tiles([128] * 8, ctx=ctx)
    ctx.close()


def test_tune_writes_and_reads_its_cache(tmp_path):
    probs = to_dev(make_set(WELL_POSED, seed0=2900))
    before = [(W.clone(), H.clone()) for _, W, H, _ in probs]
    buckets = {nb.batch_bucket(V.shape[0], V.shape[1], W.shape[1], beta) for V, W, H, beta in probs}
    assert len(buckets) >= 2
    cache = str(tmp_path / "tiles.txt")
    with open(cache, "w") as f:
        f.write("a line of another tool\n")
    ctx = nb.Context(0)
    print("[tune] first call", flush=True)
    tiles, ms, hit = nb.tune(probs, "joint", iters=1, cache=cache, ctx=ctx)
    assert not hit and ms > 0 and len(tiles) == nb.BATCH_BUCKETS
    assert all(t in (4, 8, 16, 32, 64, 128, 256) for t in tiles)
    for (W0, H0), (_, W, H, _) in zip(before, probs):
        assert torch.equal(W0, W) and torch.equal(H0, H)
    assert nb.get_batch_tiles(ctx) == tiles
    lines = open(cache).read().splitlines()
    assert lines[0] == "a line of another tool"
    entries = [l.split() for l in lines if l.startswith("nmf_tune ")]
    assert len(entries) == 1 and entries[0][1] == "2"
    mask = int(entries[0][6], 16)
    assert mask == sum(1 << b for b in buckets)
    assert [int(x) for x in entries[0][7:7 + nb.BATCH_BUCKETS]] == tiles
    # a second context reads the entry and measures nothing
    ctx2 = nb.Context(0)
    tiles2, ms2, hit2 = nb.tune(probs, "joint", iters=1, cache=cache, ctx=ctx2)
    assert hit2 and tiles2 == tiles and abs(ms2 - ms) <= 1e-6 * ms + 1e-6
    assert nb.get_batch_tiles(ctx2) == tiles
    # another mode is another key: a second entry, the first one kept
    _, _, hit3 = nb.tune(probs, "alternating", iters=1, cache=cache, ctx=ctx2)
    assert not hit3
    lines = open(cache).read().splitlines()
    assert lines[0] == "a line of another tool"
    assert len([l for l in lines if l.startswith("nmf_tune ")]) == 2
    # a problem in a bucket the entry does not cover: that bucket is tuned, the
    # others keep the cached tiles
    extra = to_dev(make_set([(5000, 300, 60, 1.0)], seed0=2950))
    b_extra = nb.batch_bucket(5000, 300, 60, 1.0)
    assert b_extra not in buckets
    tiles4, _, hit4 = nb.tune(probs + extra, "joint", iters=1, cache=cache, ctx=ctx2)
    assert not hit4
    assert all(tiles4[b] == tiles[b] for b in buckets)
    entries = [l.split() for l in open(cache).read().splitlines() if l.startswith("nmf_tune ") and l.split()[4] == "1"]
    assert len(entries) == 1 and int(entries[0][6], 16) == mask | (1 << b_extra)
    # an unwritable cache path is reported
    with pytest.raises(nb.NmfError) as e:
        nb.tune(probs, "joint", iters=1, cache=str(tmp_path / "no_such_dir" / "t.txt"), ctx=nb.Context(0))
    assert e.value.status == 10
    ctx.close()
    ctx2.close()
