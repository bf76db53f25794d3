"""The select entry point that allocates nothing
(rt_range_select_device_noalloc, workspace in the library's fixed device
scratch) against rt_range_select_device with a caller workspace, and against
the CPU oracle: two calls in a row, the second with a smaller input, so the
scratch left by the first call must not leak into the second."""

import sys

import numpy as np
import pytest

import oracle
import rtgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_noalloc_matches_device_select():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    import paper_2309_16913_amd as rt
    ora = oracle.get()
    r = rtgen.clustered_rects(400_000, 16, 0.02, 1e-3, 601)
    t = rt.build_str(r, 32, "soa")
    t.set_split(4)   # split items exercise more of the workspace
    ot = ora.build_str(r, 32)
    s = torch.cuda.current_stream().cuda_stream
    for k, nq in enumerate((20_000, 3_000)):
        say(f"case noalloc call {k} nq={nq}")
        q = rtgen.windows_loguniform(nq, 1e-7, 1e-3, 602 + k)
        wo, wi = ora.select(ot, q)
        total = int(wo[-1])
        assert rt.select_workspace_bytes(nq, total + 64) <= rt.NOALLOC_SCRATCH_BYTES
        dq = torch.from_numpy(q).cuda()
        # reference: the entry point with a caller workspace
        off_ref = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
        ids_ref = torch.empty(total + 64, dtype=torch.int32, device="cuda")
        st_ref = torch.zeros(2, dtype=torch.int64, device="cuda")
        wb = rt.select_workspace_bytes(nq, total + 64)
        work = torch.empty(wb, dtype=torch.uint8, device="cuda")
        rt.range_select_device(t, dq.data_ptr(), nq, off_ref.data_ptr(), ids_ref.data_ptr(), total + 64,
                               work.data_ptr(), wb, st_ref.data_ptr(), s)
        off = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
        ids = torch.full((total + 64,), -3, dtype=torch.int32, device="cuda")
        st = torch.full((2,), 99, dtype=torch.int64, device="cuda")
        rt.range_select_device_noalloc(t, dq.data_ptr(), nq, off.data_ptr(), ids.data_ptr(), total + 64,
                                       st.data_ptr(), s)
        torch.cuda.synchronize()
        assert st.cpu().tolist() == [total, 0] and st_ref.cpu().tolist() == [total, 0]
        assert torch.equal(off, off_ref)
        assert torch.equal(ids[:total], ids_ref[:total])
        assert bool((ids[total:] == -3).all().item()), "wrote past the result"
        assert np.array_equal(off.cpu().numpy().astype(np.uint64), wo)
        assert np.array_equal(ids[:total].cpu().numpy().view(np.uint32), wi)
    # an undersized output: reported in the status words, ids untouched
    q = rtgen.windows_loguniform(500, 1e-5, 1e-3, 610)
    wo, _ = ora.select(ot, q)
    dq = torch.from_numpy(q).cuda()
    off = torch.empty(501, dtype=torch.int64, device="cuda")
    ids = torch.full((8,), -3, dtype=torch.int32, device="cuda")
    st = torch.zeros(2, dtype=torch.int64, device="cuda")
    rt.range_select_device_noalloc(t, dq.data_ptr(), 500, off.data_ptr(), ids.data_ptr(), 8, st.data_ptr(), s)
    torch.cuda.synchronize()
    assert int(wo[-1]) > 8
    assert st.cpu().tolist() == [int(wo[-1]), 1] and bool((ids == -3).all().item())
    # sizes beyond the fixed scratch are refused on the host, nothing enqueued
    with pytest.raises(rt.RTError) as ex:
        rt.range_select_device_noalloc(t, dq.data_ptr(), 500, off.data_ptr(), ids.data_ptr(), 1 << 26,
                                       st.data_ptr(), s)
    assert ex.value.code == rt.RT_EINVAL and "scratch" in str(ex.value)
