"""C-ABI checks that need no GPU: exported symbols, host-side argument
validation, tuning, workspace sizing and the server's admission logic (fake
executor)."""
import ctypes
import os
import re
import time

import pytest

from paper_1606_08766_amd import rsort as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "rsort.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rsort_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_header_function():
    L = R.lib()
    names = header_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(L, name), name
    assert sorted(names) == sorted(R.EXPORTS)


def test_host_validation_without_gpu():
    L = R.lib()
    vp = ctypes.c_void_p
    # n == 0 is a no-op, unknown key type is rejected, NULL pointers rejected
    assert L.rsort_plain(1, None, 0, None, None, None, 0, None) == R.OK
    assert L.rsort_plain(7, vp(16), 10, vp(4096), None, vp(1 << 20), 1 << 20, None) == R.EINVAL
    assert L.rsort_plain(1, None, 10, vp(4096), None, vp(1 << 20), 1 << 20, None) == R.EINVAL
    assert L.rsort_plain(1, vp(4096), 1 << 32, vp(1 << 40), None, vp(1 << 41), 1 << 20, None) == R.EINVAL
    # overlapping input and output
    assert L.rsort_plain(1, vp(4096), 100, vp(4096 + 8), None, vp(1 << 30), 1 << 20, None) == R.EINVAL
    # workspace too small
    need = R.plain_workspace_bytes(1, 100000)
    assert L.rsort_plain(1, vp(1 << 30), 100000, vp(1 << 31), None, vp(1 << 33), need - 1, None) == R.ENOMEM
    # segmented: empty call, missing offsets, mismatched payload pointers
    assert L.rsort_segmented(1, None, None, None, 0, 0, None, None, None, None, 0, None) == R.OK
    assert L.rsort_segmented(1, vp(4096), None, None, 3, 10, vp(1 << 20), None, None, vp(1 << 30), 1 << 20,
                             None) == R.EINVAL
    assert L.rsort_segmented(1, vp(4096), vp(1 << 16), vp(1 << 18), 1, 10, vp(1 << 20), None, None, vp(1 << 30),
                             1 << 20, None) == R.EINVAL
    assert L.rsort_median_tree(None, 0, None, 0, 3, None, 1, None, None, 0, None) == R.EINVAL
    assert R.strerror(R.ENOTFOUND) == "unknown ticket"


def test_rquick_mw_host_validation_without_gpu():
    """The hypercube quicksort's shape rules: u32/f32 keys only, 1 <= log2_p
    <= 8, even window 2..16, at most 8192 keys per PE."""
    L = R.lib()
    vp = ctypes.c_void_p
    ws = 1 << 30

    def call(kt=R.U32, n=1000, log2_p=2, k=16, tb=1, kin=vp(1 << 20), kout=vp(1 << 24), wsb=ws):
        return L.rsort_rquick_mw(kt, kin, n, log2_p, k, tb, 1, kout, None, None, vp(1 << 32), wsb, None)

    assert call(n=0) == R.OK
    assert call(kt=R.U64) == R.EINVAL
    assert call(log2_p=0) == R.EINVAL and call(log2_p=9) == R.EINVAL
    assert call(k=3) == R.EINVAL and call(k=0) == R.EINVAL and call(k=18) == R.EINVAL
    assert call(n=8192 * 4 + 1, log2_p=2) == R.EINVAL  # a PE part above 8192 keys
    assert call(tb=3) == R.EINVAL and call(tb=-1) == R.EINVAL
    assert call(kin=None) == R.EINVAL
    assert call(kout=vp((1 << 20) + 8)) == R.EINVAL  # overlapping input and output
    assert call(wsb=R.rquick_mw_workspace_bytes(1000, 2) - 1) == R.ENOMEM
    assert R.rquick_mw_workspace_bytes(8192 * 4, 2) > 2 * 8 * 8192 * 4
    assert R.rquick_mw_workspace_bytes(8192 * 4 + 1, 2) == 0


def test_workspace_sizes_monotone():
    for kt in (R.U32, R.U64, R.F32):
        prev = 0
        for n in (1, 100, 12288, 12289, 1 << 20, 1 << 24):
            b = R.plain_workspace_bytes(kt, n)
            assert b >= prev
            prev = b
    assert R.plain_workspace_bytes(5, 10) == 0
    assert R.segmented_workspace_bytes(R.U64, 1 << 20, 1000, True) > R.segmented_workspace_bytes(R.U64, 1 << 20, 1000,
                                                                                                   False)
    # 2^28 u64 keys: two ping-pong buffers of 12 B/key plus small tables
    b = R.plain_workspace_bytes(R.U64, 1 << 28)
    assert 6 << 30 < b < 8 << 30


def test_tuning_roundtrip():
    t0 = R.get_tuning()
    with R.tuned(oversample=8, tile_log2=13, force_fallback=1):
        t = R.get_tuning()
        assert t.oversample == 8 and t.tile_log2 == 13 and t.force_fallback == 1
    t1 = R.get_tuning()
    assert (t1.oversample, t1.tile_log2, t1.force_fallback) == (t0.oversample, t0.tile_log2, t0.force_fallback)
    with pytest.raises(R.RsortError):
        R.set_tuning(tile_log2=11)
    with pytest.raises(R.RsortError):
        R.set_tuning(oversample=33)


# ---------------------------------------------------------------- server (fake executor, host only)
def fake_req(s, n, kt=R.U64, bad=False):
    return s.submit(kt, 0xBAD if bad else 0x1000, n, 0x100000, None)


LARGE = 1 << 21  # above the small-request lane


def test_server_admission_budget_and_tickets():
    per = R.Server.request_bytes(R.U64, LARGE)
    assert per >= LARGE * 24  # two (key, index) buffers at least
    budget = 10 * per  # arena for 10 requests of 2^21 u64 keys
    with R.Server(device=-1, hbm_budget_bytes=budget, max_inflight=4) as s:
        with pytest.raises(R.RsortError) as e:
            fake_req(s, budget)  # alone larger than the budget
        assert e.value.code == R.ENOMEM
        tickets = [fake_req(s, LARGE) for _ in range(12)]
        assert len(set(tickets)) == 12
        peak = 0
        while True:
            c = s.counters()
            assert c["bytes_in_use"] <= budget
            assert c["running"] <= 4
            peak = max(peak, c["running"])
            if c["finished"] == 12:
                break
            time.sleep(0.0002)
        assert peak >= 2  # requests overlap
        for t in tickets:
            rc, r = s.poll(t)
            assert rc == R.OK and r.t_submit_ns <= r.t_start_ns <= r.t_done_ns
        assert s.poll(123456)[0] == R.ENOTFOUND
        assert s.release(tickets[0]) == R.OK
        assert s.poll(tickets[0])[0] == R.ENOTFOUND


def test_server_fifo_and_memory_wait():
    per = R.Server.request_bytes(R.U64, LARGE)
    with R.Server(device=-1, hbm_budget_bytes=2 * per, max_inflight=8) as s:
        ts = [fake_req(s, LARGE) for _ in range(6)]
        starts = []
        for t in ts:
            rc, r = s.wait(t, 5000)
            assert rc == R.OK
            starts.append(r.t_start_ns)
        assert starts == sorted(starts)  # admitted in arrival order
        # at most two fit the budget at a time: the third starts after the first ends
        r0 = s.poll(ts[0])[1]
        r2 = s.poll(ts[2])[1]
        assert r2.t_start_ns >= r0.t_done_ns


def test_server_error_goes_to_its_ticket_only():
    with R.Server(device=-1, hbm_budget_bytes=1 << 34, max_inflight=1) as s:
        good1 = fake_req(s, 1000)
        bad = fake_req(s, 1000, bad=True)
        good2 = fake_req(s, 1000)
        assert s.wait(good1, 5000)[0] == R.OK
        assert s.wait(bad, 5000)[0] == R.EDEVICE
        assert s.wait(good2, 5000)[0] == R.OK
        zero = s.submit(R.U32, 0, 0, 0, None)
        assert s.poll(zero)[0] == R.OK


def test_server_packs_small_requests():
    # small requests queued behind a running batch are packed into one launch,
    # grouped by key type, and each keeps its own ticket and status
    with R.Server(device=-1, hbm_budget_bytes=1 << 34, max_inflight=2) as s:
        kts = [R.U32, R.U64, R.F32]
        ts = [(fake_req(s, 5000 + i, kt=kts[i % 3], bad=(i == 77)), kts[i % 3], i) for i in range(300)]
        by_start = {}
        for t, kt, i in ts:
            rc, r = s.wait(t, 5000)
            assert rc == (R.EDEVICE if i == 77 else R.OK)
            assert 1 <= r.batch_size <= 1024
            by_start.setdefault(r.t_start_ns, []).append((kt, r.batch_size))
        assert max(len(v) for v in by_start.values()) > 1  # some batch packed several requests
        for group in by_start.values():
            assert len({kt for kt, _ in group}) == 1  # one key type per batch
            assert all(b == len(group) for _, b in group)
        c = s.counters()
        assert c["finished"] == 300 and c["running"] == 0 and c["bytes_in_use"] == 0  # arena fully returned


def test_server_arena_fragmentation_and_reuse():
    # mixed sizes through a small arena: never over budget, every request
    # finishes, and the arena coalesces back to one free block
    sizes = [LARGE, 3 * LARGE, LARGE + 7, 5000, 2 * LARGE, 70000, LARGE, 1 << 20]
    budget = R.Server.request_bytes(R.U64, 3 * LARGE) + R.Server.request_bytes(R.U64, LARGE)
    with R.Server(device=-1, hbm_budget_bytes=budget, max_inflight=6) as s:
        ts = [fake_req(s, sizes[i % len(sizes)]) for i in range(64)]
        while s.counters()["finished"] < 64:
            assert s.counters()["bytes_in_use"] <= budget
            time.sleep(0.0002)
        assert all(s.poll(t)[0] == R.OK for t in ts)
        assert s.counters()["bytes_in_use"] == 0
    assert R.Server.request_bytes(R.U64, 0) == 0 and R.Server.request_bytes(9, 10) == 0


def test_server_rejects_bad_requests():
    with R.Server(device=-1, hbm_budget_bytes=1 << 30, max_inflight=2) as s:
        with pytest.raises(R.RsortError):
            s.submit(9, 0x1000, 10, 0x2000, None)
        with pytest.raises(R.RsortError):
            s.submit(R.U32, 0, 10, 0x2000, None)
    with pytest.raises(R.RsortError):
        R.Server(device=-1, hbm_budget_bytes=1 << 30, max_inflight=0)


# ---------------------------------------------------------------- autotuner (host logic)
def test_autotune_threshold_choice():
    from paper_1606_08766_amd import autotune as A
    # merge fastest everywhere: RFIS and RQuick turned off
    t = {(b, "merge"): 1.0 for b in A.CLASS_BOUNDS}
    t.update({(b, "rfis"): 2.0 for b in A.RFIS_BOUNDS})
    t.update({(b, "rquick"): 3.0 for b in A.RQUICK_BOUNDS})
    assert A.choose_thresholds(t)[:2] == (1, 1)
    # RFIS wins up to 256, RQuick at 2048 and 3072: thresholds express exactly that
    t[(64, "rfis")] = t[(256, "rfis")] = 0.5
    t[(2048, "rquick")] = t[(3072, "rquick")] = 0.5
    rf, rq, total = A.choose_thresholds(t)
    assert (rf, rq) == (256, 3072)
    assert total == pytest.approx(0.5 * 4 + 1.0 * (len(A.CLASS_BOUNDS) - 4))
    # a non-contiguous winner set is approximated by the cheapest contiguous choice
    t[(256, "rfis")] = 5.0
    assert A.choose_thresholds(t)[0] == 64
    assert A.algo_for(64, 256, 3072) == "rfis" and A.algo_for(4096, 256, 3072) == "merge"
    assert A.algo_for(2048, 256, 3072) == "rquick"


def test_autotune_save_load_roundtrip(tmp_path):
    from paper_1606_08766_amd import autotune as A
    saved = R.get_tuning()
    try:
        res = {"rfis_max": 64, "rquick_max": 2048, "tile_log2": 13, "oversample": 16, "target": 3072}
        p = str(tmp_path / "t.json")
        A.save(res, p)
        A.load(p)
        t = R.get_tuning()
        assert (t.rfis_max, t.rquick_max, t.tile_log2, t.oversample, t.target) == (64, 2048, 13, 16, 3072)
    finally:
        R.set_tuning(**{f: getattr(saved, f) for f, _ in R.Tuning._fields_})


def test_binding_rejects_signed_keys_and_bad_side_tensors():
    """Signed integer keys would be ordered by their unsigned bit pattern
    (negative after positive), so the binding refuses them unless the caller
    names the unsigned key type on purpose; side tensors handed to the C ABI
    as raw pointers are checked for size and element type first."""
    import torch

    for dt in (torch.int32, torch.int64):
        x = torch.tensor([-3, 2, -1, 5], dtype=dt)
        with pytest.raises(TypeError):
            R.sort(x)
        with pytest.raises(TypeError):
            R.segmented_sort(x, torch.tensor([0, 4], dtype=torch.int64))
    # an explicit key type of the wrong width is refused as well
    with pytest.raises(TypeError):
        R._kt(torch.zeros(4, dtype=torch.int32), R.U64)
    assert R._kt(torch.zeros(4, dtype=torch.int64), R.U64) == R.U64
    assert R._kt(torch.zeros(4, dtype=torch.float32)) == R.F32
    cpu = torch.device("cpu")
    with pytest.raises(ValueError):  # not a device tensor
        R._require_like(torch.zeros(4, dtype=torch.uint32), "perm_out", cpu, 4, 4, R._U32_LIKE)


def test_noalloc_refuses_sizes_beyond_its_scratch_without_gpu():
    """rsort_plain_noalloc checks its size limit (64 MiB of workspace) before
    any device call."""
    n = 1 << 24
    assert R.plain_workspace_bytes(R.U64, n) > (64 << 20)
    rc = R.lib().rsort_plain_noalloc(R.U64, ctypes.c_void_p(16), n, ctypes.c_void_p(1 << 40), None, None)
    assert rc == R.ENOMEM
    assert R.lib().rsort_plain_noalloc(7, None, 5, None, None, None) == R.EINVAL
    assert R.lib().rsort_plain_noalloc(R.U32, None, 0, None, None, None) == R.OK
