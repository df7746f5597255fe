"""lev_batch_noalloc (workspace in the library's fixed device array) against
lev_batch (caller workspace), through the C ABI, on two calls in a row, the
second on a smaller input (GPU)."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import pyoracle as orc
from paper_2601_15458_amd import msadp, synth

pytestmark = pytest.mark.gpu


def _noalloc(A, B, ia, ib):
    f = msadp.lib().lev_batch_noalloc
    dev = A.codes.device
    ia_d = torch.as_tensor(np.ascontiguousarray(ia, np.int32), device=dev)
    ib_d = torch.as_tensor(np.ascontiguousarray(ib, np.int32), device=dev)
    out = torch.empty(max(len(ia), 1), dtype=torch.uint16, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    sa, sb = A.struct(), B.struct()
    rc = f(C.byref(sa), C.byref(sb), ia_d.data_ptr(), ib_d.data_ptr(), len(ia), out.data_ptr(),
           st.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert rc == 0, msadp.lib().msa_strerror(rc)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    return out[: len(ia)].cpu().numpy().astype(np.int64)


def test_noalloc_matches_lev_batch_twice_second_smaller():
    cases = [
        # one pattern per lane (DNA up to 512), 150,000 pairs
        (11, 3000, 50, 512, 150_000),
        # shared patterns (up to 1500 rows), fewer sequences and pairs
        (12, 120, 0, 1500, 4000),
    ]
    for seed, n, lo, hi, n_pairs in cases:
        codes, off = synth.random_set(seed, n, lo, hi, 4)
        A = msadp.to_device(codes, off, 4)
        rng = np.random.default_rng(seed)
        ia = rng.integers(0, n, n_pairs)
        ib = rng.integers(0, n, n_pairs)
        want = msadp.lev_batch(A, A, ia, ib).cpu().numpy().astype(np.int64)
        got = _noalloc(A, A, ia, ib)
        assert (got == want).all(), (seed, np.flatnonzero(got != want)[:5])
        pick = rng.choice(n_pairs, 2000, replace=False)
        assert (got[pick] == orc.lev_pairs(codes, off, codes, off, ia[pick], ib[pick])).all()


def test_noalloc_rejects_inputs_beyond_its_array():
    codes, off = synth.random_set(13, 50, 10, 100, 4)
    A = msadp.to_device(codes, off, 4)
    f = msadp.lib().lev_batch_noalloc
    sa = A.struct()
    assert msadp.lib().lev_workspace_bytes(C.byref(sa), C.byref(sa), 1 << 24) > \
        msadp.NOALLOC_SCRATCH_BYTES
    # 2^24 pairs need more than 64 MiB of workspace: refused on the host
    # before anything is read or launched (the pair pointers are never used)
    dummy = torch.zeros(1, dtype=torch.int32, device=A.codes.device)
    rc = f(C.byref(sa), C.byref(sa), dummy.data_ptr(), dummy.data_ptr(), 1 << 24,
           dummy.data_ptr(), None, torch.cuda.current_stream().cuda_stream)
    assert rc == msadp.MSA_ENOSPC
