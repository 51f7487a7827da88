"""The continuous-batching server: requests of mixed kinds, shapes and error
bounds, submitted while others run, admitted by HBM footprint and run on
overlapping slots.  Every served result must be byte for byte what the
single-field calls give for that request alone (and, for compressions, the
oracle's archive)."""
from __future__ import annotations

import threading
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _pool():
    from synth import fields
    xs = [fields.hurricane3d((40, 64, 80), seed=1), fields.hurricane3d((17, 33, 130), seed=2),
          fields.fourier2d((300, 410), seed=3), fields.fourier2d((45, 2000), seed=4),
          fields.particles1d(200003, seed=5, shuffle_block=256), fields.particles1d(4097, seed=6, shuffle_block=256),
          fields.hurricane3d((64, 64, 64), seed=7), fields.fourier2d((1, 3), seed=8)]
    return xs


@pytest.fixture(scope="module")
def case():
    import torch
    from paper_2007_09625_amd import dqz
    xs = _pool()
    ts = [torch.from_numpy(x).cuda() for x in xs]
    ebs = [1e-4, 1e-3, 1e-2, 1e-5]
    reqs = []   # (kind, field index, eb)
    for k in range(48):
        reqs.append(("c" if k % 3 else "d", k % len(xs), ebs[(k // len(xs)) % len(ebs)]))
    ctx = dqz.Context(0)
    plain = {}
    for kind, i, eb in reqs:
        if (i, eb) not in plain:
            c = ctx.compress(ts[i], eb)
            plain[(i, eb)] = (c, ctx.decompress(c).clone())
    torch.cuda.synchronize()
    return xs, ts, reqs, plain


def _serve(dqz, ts, reqs, plain, slots, budget, stagger=False):
    """Submit every request (the second half from another thread while the
    first half runs when stagger); return outputs in request order."""
    import torch
    sv = dqz.Server(0, slots=slots, workspace=256 << 20, budget=budget)
    outs, tickets = [None] * len(reqs), [None] * len(reqs)

    def submit(lo, hi):
        for k in range(lo, hi):
            kind, i, eb = reqs[k]
            if kind == "c":
                bound, _ = dqz.dqz_compress_bound(tuple(ts[i].shape), dqz.make_params(eb))
                out = torch.empty(bound, dtype=torch.uint8, device="cuda")
                tickets[k] = sv.submit_compress(ts[i], eb, out)
            else:
                c = plain[(i, eb)][0]
                out = torch.empty_like(ts[i])
                tickets[k] = sv.submit_decompress(c.archive, c.nbytes, c.header, out)
            outs[k] = out

    half = len(reqs) // 2
    submit(0, half)
    if stagger:
        th = threading.Thread(target=submit, args=(half, len(reqs)))
        time.sleep(0.002)
        th.start()
        th.join()
    else:
        submit(half, len(reqs))
    comps = [sv.wait(t) for t in tickets]
    stats = sv.stats()
    sv.close()
    return outs, comps, stats


def _check(reqs, plain, outs, comps):
    import torch
    for k, ((kind, i, eb), out, c) in enumerate(zip(reqs, outs, comps)):
        assert c.status == 0, (k, c.status)
        ref, ref_y = plain[(i, eb)]
        if kind == "c":
            assert c.output_bytes == ref.nbytes, k
            assert torch.equal(out[:c.output_bytes], ref.archive), k
            assert bytes(c.header) == ref.header, k
        else:
            assert torch.equal(out.view(torch.int32), ref_y.view(torch.int32)), k
        assert c.t_submit_us <= c.t_admit_us <= c.t_done_us


def test_served_results_equal_alone_and_in_the_mix(case):
    import oracle
    from paper_2007_09625_amd import dqz
    xs, ts, reqs, plain = case
    # in the mix: 4 slots, a budget large enough for several at once, the
    # second half arriving while the first half runs
    outs, comps, stats = _serve(dqz, ts, reqs, plain, slots=4, budget=1 << 34, stagger=True)
    _check(reqs, plain, outs, comps)
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert stats["max_running"] >= 2          # requests overlapped on the device
    # alone: one slot, every request by itself
    outs1, comps1, stats1 = _serve(dqz, ts, reqs, plain, slots=1, budget=1 << 34)
    _check(reqs, plain, outs1, comps1)
    assert stats1["max_running"] == 1
    # and the compressions are the oracle's archives
    seen = set()
    for (kind, i, eb), out, c in zip(reqs, outs, comps):
        if kind == "c" and (i, eb) not in seen and len(seen) < 6:
            seen.add((i, eb))
            assert np.array_equal(out[:c.output_bytes].cpu().numpy(), oracle.compress(xs[i], eb))


def test_admission_by_footprint(case):
    """With a budget below any single footprint every request runs alone;
    with a budget of about two footprints at most a few run together and
    the summed footprint of the running ones stays within the budget."""
    from paper_2007_09625_amd import dqz
    xs, ts, reqs, plain = case
    sub = [r for r in reqs if r[1] in (0, 6)][:12]     # the two largest 3D fields
    outs, comps, stats = _serve(dqz, ts, sub, plain, slots=4, budget=1 << 20)
    _check(sub, plain, outs, comps)
    assert stats["max_running"] == 1
    fp = max(c.footprint for c in comps)
    outs, comps, stats = _serve(dqz, ts, sub, plain, slots=4, budget=2 * fp + fp // 2)
    _check(sub, plain, outs, comps)
    assert stats["max_in_flight_bytes"] <= 2 * fp + fp // 2


def test_overflow_runs_again_with_reported_workspace():
    """Every element an outlier and most of them patches too (values near
    2^27 quantization steps: random deltas far outside the cap, and d° above
    2^24 is not exact in fp32): about two exception records per element
    overflow the request's first workspace (room for one per element); the
    server runs it again with the size the device reported and the archive
    is the oracle's."""
    import torch
    import oracle
    from paper_2007_09625_amd import dqz
    rng = np.random.default_rng(31)
    x = rng.uniform(-2.6e5, 2.6e5, 20000).astype(np.float32)
    t = torch.from_numpy(x).cuda()
    sv = dqz.Server(0, slots=2, workspace=64 << 20, budget=1 << 30)
    bound, _ = dqz.dqz_compress_bound(tuple(x.shape), dqz.make_params(1e-3, dqz.DQZ_EB_ABS))
    out = torch.empty(bound, dtype=torch.uint8, device="cuda")
    c = sv.wait(sv.submit_compress(t, 1e-3, out, mode="abs"))
    stats = sv.stats()
    sv.close()
    ref = oracle.compress(x, 1e-3, oracle.EB_ABS)
    import archive_util as au
    h = au.header(ref)
    assert h["n_out"] + h["n_patch"] > x.size          # more records than the first workspace holds
    assert c.status == 0 and stats["retried"] >= 1
    assert np.array_equal(out[:c.output_bytes].cpu().numpy(), ref)


def test_submit_rejects_what_can_never_run():
    import torch
    from paper_2007_09625_amd import dqz
    sv = dqz.Server(0, slots=1, workspace=1 << 20, budget=1 << 30)
    t = torch.zeros((128, 128, 128), dtype=torch.float32, device="cuda")
    out = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(dqz.DqzError) as e:
        sv.submit_compress(t, 1e-3, out)      # workspace above the 1 MiB arena
    assert e.value.status == dqz.DQZ_ENOMEM
    with pytest.raises(dqz.DqzError) as e:
        sv.wait(12345)
    assert e.value.status == dqz.DQZ_EINVAL
    sv.close()
