"""Serving form on the GPU: continuous batching of many streams of different
N and T. Each stream's outputs must equal the oracle's stream PPF, and the
same stream must give the same spectra alone and in the mix."""

from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1411_3656_amd import ppf, signals

pytestmark = pytest.mark.gpu
TOL = 1e-5
PLANS = [(256, 8), (1024, 8), (1024, 16), (4096, 16)]


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rel_err(got, ref):
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    return float(np.max(np.abs(got - ref))) / rms


class Workload:
    """Streams with pre-generated chunk inputs (host and device) and outputs."""

    def __init__(self, torch, n_streams, seed, max_spectra=40, chunks_per_stream=6):
        rng = np.random.default_rng(seed)
        self.torch = torch
        self.coeffs = {}
        self.streams = []
        for i in range(n_streams):
            n, taps = PLANS[int(rng.integers(len(PLANS)))] if i else PLANS[1]
            lens = [int(v) for v in rng.integers(1, max_spectra + 1, chunks_per_stream)]
            if n == 4096:
                lens = [min(v, 12) for v in lens]
            x = signals.complex_gaussian(sum(lens) * n, 1.0, seed=seed * 1000 + i)
            chunks, at = [], 0
            for s in lens:
                chunks.append(x[at * n:(at + s) * n])
                at += s
            dev_in = [torch.from_numpy(c).cuda() for c in chunks]
            self.streams.append(dict(n=n, taps=taps, lens=lens, chunks=chunks, dev_in=dev_in))
        for n, taps in PLANS:
            rng2 = np.random.default_rng(n * 7 + taps)
            self.coeffs[(n, taps)] = rng2.standard_normal(taps * n).astype(np.float32)

    def run(self, server, plans, which, order_seed):
        """Push the chunks of streams `which`, interleaved across streams in a
        random order (in order within a stream); return outputs per stream."""
        torch = self.torch
        handles = {}
        outs = {}
        for k in which:
            st = self.streams[k]
            handles[k] = ppf.ppf_server_open_stream(server, plans[(st["n"], st["taps"])].handle)
            outs[k] = [torch.full((s, st["n"]), float("nan"), dtype=torch.complex64, device="cuda")
                       for s in st["lens"]]
        cursor = {k: 0 for k in which}
        rng = np.random.default_rng(order_seed)
        live = list(which)
        tags = []
        while live:
            k = live[int(rng.integers(len(live)))]
            i = cursor[k]
            st = self.streams[k]
            tag = k * 1000 + i
            ppf.ppf_stream_push(handles[k], st["dev_in"][i], outs[k][i], st["lens"][i], tag=tag)
            tags.append(tag)
            cursor[k] += 1
            if cursor[k] == len(st["lens"]):
                live.remove(k)
        ppf.ppf_server_drain(server, 120.0)
        done = []
        while True:
            got = ppf.ppf_server_poll(server)
            if not got:
                break
            done.extend(got)
        assert sorted(done) == sorted(tags)
        for k in which:
            ppf.ppf_stream_destroy(handles[k])
        torch.cuda.synchronize()
        return {k: np.concatenate([o.cpu().numpy() for o in outs[k]]) for k in which}


def _plans(coeffs):
    return {key: ppf.Plan(key[0], key[1], h) for key, h in coeffs.items()}


def test_mix_matches_oracle_and_alone():
    """Twelve streams of four plans pushed interleaved through one server
    match the oracle's stream form, and every stream, run alone in a fresh
    server, gives bit-identical spectra to its spectra in the mix."""
    torch = _torch()
    wl = Workload(torch, n_streams=12, seed=5)
    plans = _plans(wl.coeffs)
    srv = ppf.ppf_server_create(1 << 32, 2)
    try:
        mix = wl.run(srv, plans, list(range(12)), order_seed=1)
        stats = ppf.ppf_server_get_stats(srv)
        p50, p99, gbps = ppf.ppf_server_stats(srv)
    finally:
        ppf.ppf_server_destroy(srv)
    assert stats["chunks_done"] == sum(len(s["lens"]) for s in wl.streams)
    assert stats["batches"] >= 1 and stats["p99_us"] >= stats["p50_us"] > 0
    assert (p50, p99) == (stats["p50_us"], stats["p99_us"]) and gbps > 0
    for k, st in enumerate(wl.streams):
        h = wl.coeffs[(st["n"], st["taps"])]
        ref = np.concatenate(oracle.ppf_stream(st["chunks"], h, st["n"], st["taps"]))
        assert mix[k].shape == ref.shape
        err = rel_err(mix[k], ref)
        print(f"stream {k} N={st['n']} T={st['taps']} chunks={st['lens']} err={err:.2e}")
        assert err <= TOL, (k, err)
    for k in range(12):
        srv = ppf.ppf_server_create(1 << 32, 2)
        try:
            alone = wl.run(srv, plans, [k], order_seed=2 + k)
        finally:
            ppf.ppf_server_destroy(srv)
        assert np.array_equal(alone[k], mix[k]), k
    for p in plans.values():
        p.close()


def _fixed_bytes():
    probe = ppf.ppf_server_create(1 << 32, 2)
    fixed = ppf.ppf_server_get_stats(probe)["state_bytes_used"]   # the server's own buffers
    ppf.ppf_server_destroy(probe)
    return fixed


def test_budget_admission_queues_and_releases():
    torch = _torch()
    wl = Workload(torch, n_streams=1, seed=9, chunks_per_stream=1)
    plans = _plans(wl.coeffs)
    state = 2 * (8 - 1) * 1024 * 8 + 4096          # two history buffers + bookkeeping
    srv = ppf.ppf_server_create(_fixed_bytes() + 2 * state + 100, 2)
    try:
        key = (1024, 8)
        a = ppf.ppf_server_open_stream(srv, plans[key].handle)
        b = ppf.ppf_server_open_stream(srv, plans[key].handle)
        with pytest.raises(ppf.PPFError) as ei:
            ppf.ppf_server_open_stream_ex(srv, plans[key].handle, ppf.PPF_OPEN_NOWAIT)
        assert ei.value.status == ppf.PPF_ERR_BUDGET
        c = ppf.ppf_server_open_stream(srv, plans[key].handle)     # waits in line
        assert not ppf.ppf_server_stream_admitted(c)
        x = signals.complex_gaussian(20 * 1024, 1.0, seed=77)
        xd = torch.from_numpy(x).cuda()
        od = torch.empty((20, 1024), dtype=torch.complex64, device="cuda")
        ppf.ppf_server_submit(c, xd, od, 20, tag=7)      # waits with the stream
        ppf.ppf_stream_destroy(a)                         # frees budget: c is admitted
        ppf.ppf_server_drain(srv, 60.0)
        assert ppf.ppf_server_stream_admitted(c)
        assert ppf.ppf_server_poll(srv) == [7]
        ref = oracle.ppf_stream([x], wl.coeffs[key], 1024, 8)[0]
        assert rel_err(od.cpu().numpy(), ref) <= TOL
        stats = ppf.ppf_server_get_stats(srv)
        assert stats["rejected"] == 1 and stats["queued_admissions"] == 1
        ppf.ppf_stream_destroy(b)
        ppf.ppf_stream_destroy(c)
    finally:
        ppf.ppf_server_destroy(srv)
    for p in plans.values():
        p.close()


def test_state_that_can_never_fit_is_refused():
    _torch()
    plan = ppf.Plan(16384, 64, np.ones(16384 * 64, np.float32))
    srv = ppf.ppf_server_create(_fixed_bytes() + 1000, 2)
    try:
        with pytest.raises(ppf.PPFError) as ei:
            ppf.ppf_server_open_stream(srv, plan.handle)
        assert ei.value.status == ppf.PPF_ERR_BUDGET
    finally:
        ppf.ppf_server_destroy(srv)
    plan.close()


def test_close_while_waiting_drops_its_chunks():
    """A stream closed before admission leaves the line; its pushed chunks
    are dropped, so drain and destroy still return."""
    torch = _torch()
    plan = ppf.Plan(1024, 8, np.ones(8192, np.float32))
    state = 2 * 7 * 1024 * 8 + 4096
    srv = ppf.ppf_server_create(_fixed_bytes() + state + 100, 2)
    try:
        a = ppf.ppf_server_open_stream(srv, plan.handle)
        c = ppf.ppf_server_open_stream(srv, plan.handle)           # waits
        assert not ppf.ppf_server_stream_admitted(c)
        xd = torch.zeros(4 * 1024, dtype=torch.complex64, device="cuda")
        od = torch.empty_like(xd)
        for i in range(3):
            ppf.ppf_stream_push(c, xd, od, 4, tag=100 + i)
        ppf.ppf_server_close_stream(c)
        with pytest.raises(ppf.PPFError):
            ppf.ppf_stream_push(c, xd, od, 4)                       # closed
        assert ppf.ppf_server_drain(srv, 10.0) == ppf.PPF_OK
        assert ppf.ppf_server_poll(srv) == []                        # dropped, never reported
        ppf.ppf_stream_destroy(c)
        ppf.ppf_stream_destroy(a)
    finally:
        ppf.ppf_server_destroy(srv)
    plan.close()


def test_close_admits_waiting_stream_while_batches_run():
    """The budget of a closed stream is given back as soon as its own chunks
    are done, not when the GPU next goes idle: a waiting stream is admitted
    while another stream's batches are still running."""
    torch = _torch()
    plan = ppf.Plan(1024, 8, np.ones(8192, np.float32))
    state = 2 * 7 * 1024 * 8 + 4096
    srv = ppf.ppf_server_create(_fixed_bytes() + 2 * state + 100, 2)
    try:
        busy = ppf.ppf_server_open_stream(srv, plan.handle)
        a = ppf.ppf_server_open_stream(srv, plan.handle)
        c = ppf.ppf_server_open_stream(srv, plan.handle)            # waits
        assert not ppf.ppf_server_stream_admitted(c)
        spectra = 8192
        xd = torch.zeros(spectra * 1024, dtype=torch.complex64, device="cuda")
        od = torch.empty_like(xd)
        n_busy = 1500
        for i in range(n_busy):
            ppf.ppf_stream_push(busy, xd, od, spectra, tag=i)
        ppf.ppf_server_close_stream(a)
        import time
        t_end = time.time() + 10.0
        while not ppf.ppf_server_stream_admitted(c) and time.time() < t_end:
            time.sleep(0.0002)
        done_at_admission = len(ppf.ppf_server_poll(srv, 1 << 16))
        assert ppf.ppf_server_stream_admitted(c)
        print(f"waiting stream admitted after {done_at_admission} of {n_busy} busy chunks", flush=True)
        assert done_at_admission < n_busy
        ppf.ppf_server_drain(srv, 120.0)
        for h in (busy, a, c):
            ppf.ppf_stream_destroy(h)
    finally:
        ppf.ppf_server_destroy(srv)
    plan.close()


def test_chunk_larger_than_a_batch_runs_in_pieces():
    """A chunk beyond what one batch holds (N=4096, T=16 two-pass: 16384
    spectra fill the 512 MiB workspace) runs as consecutive pieces and
    reports its tag once; its spectra on both sides of the piece boundary
    and along the chunk match the oracle."""
    torch = _torch()
    n, taps = 4096, 16
    h = np.random.default_rng(31).standard_normal(taps * n).astype(np.float32)
    plan = ppf.Plan(n, taps, h)
    assert plan.path == ppf.PPF_PATH_TWO_PASS
    s_chunk = 16384 + 100
    x = signals.complex_gaussian(s_chunk * n, 1.0, seed=4242)
    xd = torch.from_numpy(x).cuda()
    od = torch.full((s_chunk, n), float("nan"), dtype=torch.complex64, device="cuda")
    srv = ppf.ppf_server_create(4 << 30, 2)
    try:
        st = ppf.ppf_server_open_stream(srv, plan.handle)
        ppf.ppf_stream_push(st, xd, od, s_chunk, tag=99)
        ppf.ppf_server_drain(srv, 120.0)
        assert ppf.ppf_server_poll(srv) == [99]
        ppf.ppf_stream_destroy(st)
    finally:
        ppf.ppf_server_destroy(srv)
    got = od.cpu().numpy()
    assert np.isfinite(got).all()
    whole = np.concatenate([np.zeros((taps - 1) * n, np.complex64), x])
    idx = sorted(set(list(range(0, s_chunk, 97)) + list(range(16384 - 20, 16384 + 20)) +
                     list(range(taps)) + [s_chunk - 1]))
    ref = oracle.ppf(whole, h, n, taps, spectra=idx)
    err = rel_err(got[idx], ref)
    print(f"N={n} T={taps} chunk of {s_chunk} spectra in pieces: max err / rms = {err:.3e}")
    assert err <= TOL
    plan.close()


def test_submit_errors():
    torch = _torch()
    plan = ppf.Plan(256, 4, np.ones(1024, np.float32))
    srv = ppf.ppf_server_create(1 << 30, 1)
    plain = ppf.ppf_stream_create(plan.handle)
    try:
        sid = ppf.ppf_server_open_stream(srv, plan.handle)
        buf = torch.zeros(8 * 256, dtype=torch.complex64, device="cuda")
        out = torch.empty_like(buf)
        with pytest.raises(ppf.PPFError) as ei:
            ppf.ppf_server_submit(plain, buf, out, 2)          # not a server stream
        assert ei.value.status == ppf.PPF_ERR_INVALID
        with pytest.raises(ppf.PPFError) as ei:
            ppf.ppf_server_submit(sid, buf, out, -1)
        assert ei.value.status == ppf.PPF_ERR_INVALID
        with pytest.raises(ppf.PPFError) as ei:
            ppf.ppf_server_submit(sid, buf.data_ptr() + 8, out, 2)
        assert ei.value.status == ppf.PPF_ERR_ALIGN
        with pytest.raises(ppf.PPFError) as ei:
            ppf.ppf_stream_get_history(sid, np.zeros(3 * 256, np.complex64))
        assert ei.value.status == ppf.PPF_ERR_UNSUPPORTED
        assert ppf.ppf_stream_position(sid) == 0
        ppf.ppf_stream_push(sid, buf, out, 2, tag=5)
        assert ppf.ppf_stream_position(sid) == 2
        ppf.ppf_server_drain(srv, 10.0)
        ppf.ppf_server_close_stream(sid)
        with pytest.raises(ppf.PPFError):
            ppf.ppf_server_submit(sid, buf, out, 2)
        ppf.ppf_stream_destroy(sid)
    finally:
        ppf.ppf_server_destroy(srv)
        ppf.ppf_stream_destroy(plain)
    with pytest.raises(ppf.PPFError) as ei:
        ppf.ppf_server_create(1 << 20, 2)
    assert ei.value.status == ppf.PPF_ERR_BUDGET
    plan.close()


def test_runs_of_short_chunks_match_oracle():
    """Chunks shorter than T-1 spectra make a chunk's history span the old
    history and earlier short chunks; several such streams, their chunks
    submitted back to back, must still give the oracle's stream PPF."""
    torch = _torch()
    rng = np.random.default_rng(23)
    plans = {}
    streams = []
    for i, (n, taps) in enumerate([(256, 16), (1024, 16), (4096, 16), (256, 8)]):
        h = rng.standard_normal(taps * n).astype(np.float32)
        plans[(n, taps)] = (ppf.Plan(n, taps, h), h)
        lens = [2, 3, 1, 5, 2, 20, 1, 1, 1, 9, 4, 17, 1, 2] if n < 4096 else [2, 3, 1, 5, 2, 6, 1, 1]
        x = signals.complex_gaussian(sum(lens) * n, 1.0, seed=900 + i)
        chunks, at = [], 0
        for s in lens:
            chunks.append(x[at * n:(at + s) * n])
            at += s
        streams.append((n, taps, lens, chunks))
    srv = ppf.ppf_server_create(1 << 32, 2)
    try:
        ids, outs, keep = [], [], []
        for n, taps, lens, chunks in streams:
            ids.append(ppf.ppf_server_open_stream(srv, plans[(n, taps)][0].handle))
            outs.append([torch.full((s, n), float("nan"), dtype=torch.complex64, device="cuda") for s in lens])
            keep.append([torch.from_numpy(c).cuda() for c in chunks])
        torch.cuda.synchronize()
        for i in range(max(len(s[2]) for s in streams)):
            for k, (n, taps, lens, chunks) in enumerate(streams):
                if i < len(lens):
                    ppf.ppf_server_submit(ids[k], keep[k][i], outs[k][i], lens[i], tag=k * 100 + i)
        ppf.ppf_server_drain(srv, 120.0)
        for k, (n, taps, lens, chunks) in enumerate(streams):
            got = np.concatenate([o.cpu().numpy() for o in outs[k]])
            ref = np.concatenate(oracle.ppf_stream(chunks, plans[(n, taps)][1], n, taps))
            err = rel_err(got, ref)
            print(f"short-chunk stream N={n} T={taps} err={err:.2e}")
            assert err <= TOL, (n, taps, err)
            ppf.ppf_stream_destroy(ids[k])
    finally:
        ppf.ppf_server_destroy(srv)
    for p, _ in plans.values():
        p.close()


def test_c5_mix_sampled_streams():
    """The serving workload's shape: 64 streams whose N in {256, 1024, 4096}
    and T in {8, 16} are drawn from each stream's seed, sinc x Hamming
    prototypes, chunks of 1..64 spectra submitted interleaved at random.
    Every chunk of 8 sampled streams is checked against the oracle's stream
    form; every output of the other streams must be finite."""
    torch = _torch()
    n_streams, chunks_per_stream = 64, 8
    streams = []
    for i in range(n_streams):
        rng = np.random.default_rng(signals.SEED_BASE + 4 + 1000 * i)
        n = int(rng.choice([256, 1024, 4096]))
        taps = int(rng.choice([8, 16]))
        lens = [int(v) for v in rng.integers(1, 65, chunks_per_stream)]
        x = signals.complex_gaussian(sum(lens) * n, 1.0, seed=signals.SEED_BASE + 4 + 1000 * i + 1)
        chunks, at = [], 0
        for s in lens:
            chunks.append(x[at * n:(at + s) * n])
            at += s
        streams.append(dict(n=n, taps=taps, lens=lens, chunks=chunks,
                            dev_in=[torch.from_numpy(c).cuda() for c in chunks]))
    shapes = sorted({(s["n"], s["taps"]) for s in streams})
    coeffs = {key: signals.design_coeffs(key[0], key[1], "hamming").astype(np.float32) for key in shapes}
    plans = _plans(coeffs)
    print(f"case C5 mix: {n_streams} streams, classes {shapes}", flush=True)
    srv = ppf.ppf_server_create(8 << 30, 2)
    try:
        ids, outs = {}, {}
        for k, st in enumerate(streams):
            ids[k] = ppf.ppf_server_open_stream(srv, plans[(st["n"], st["taps"])].handle)
            outs[k] = [torch.full((s, st["n"]), float("nan"), dtype=torch.complex64, device="cuda")
                       for s in st["lens"]]
        cursor = [0] * n_streams
        rng = np.random.default_rng(17)
        live = list(range(n_streams))
        while live:
            k = live[int(rng.integers(len(live)))]
            i = cursor[k]
            st = streams[k]
            ppf.ppf_server_submit(ids[k], st["dev_in"][i], outs[k][i], st["lens"][i], tag=k * 1000 + i)
            cursor[k] += 1
            if cursor[k] == chunks_per_stream:
                live.remove(k)
        ppf.ppf_server_drain(srv, 120.0)
        for k in range(n_streams):
            ppf.ppf_stream_destroy(ids[k])
        torch.cuda.synchronize()
    finally:
        ppf.ppf_server_destroy(srv)
        for p in plans.values():
            p.close()
    sampled = list(range(0, n_streams, n_streams // 8))
    for k, st in enumerate(streams):
        got = np.concatenate([o.cpu().numpy() for o in outs[k]])
        assert np.isfinite(got).all(), k
        if k in sampled:
            ref = np.concatenate(oracle.ppf_stream(st["chunks"], coeffs[(st["n"], st["taps"])], st["n"], st["taps"]))
            err = rel_err(got, ref)
            print(f"C5 stream {k} N={st['n']} T={st['taps']} chunks {st['lens']}: max err / rms = {err:.3e}",
                  flush=True)
            assert err <= TOL, (k, err)
