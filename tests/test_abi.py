"""The C-ABI library: loads, exports what include/msadp.h declares, and
rejects bad arguments on the host before anything is launched (no GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_2601_15458_amd import msadp

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                   "msadp.h")


def declared_functions():
    text = open(HDR).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_every_declared_symbol_is_exported():
    L = C.CDLL(msadp.LIB_PATH)
    names = declared_functions()
    assert {"lev_batch", "nw_batch", "nw_traceback", "lev_allpairs"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(msadp.SIGNATURES), "binding and header disagree"


def test_tb_bytes_closed_form():
    L = msadp.lib()
    assert L.nw_tb_bytes(0, 10) == 0 and L.nw_tb_bytes(10, 0) == 0
    for m, n in [(1, 1), (32, 7), (33, 7), (100, 50), (10000, 9000)]:
        W = (m + 31) // 32
        assert L.nw_tb_bytes(m, n) == (n + W - 1) * W * 8
        assert L.nw_tb_bytes(m, n) >= m * n // 4          # at least 2 bits per cell


def test_strerror_and_version():
    L = msadp.lib()
    assert L.msa_version() >= 1
    for code in (0, -1, -2, -3, -4):
        assert L.msa_strerror(code)


def _seqs(n=3, sigma=4, max_len=10, packed=0, codes=1, offsets=1):
    return msadp.MsaSeqs(codes, offsets, n, sigma, max_len, packed)


@pytest.mark.parametrize("kw,code", [
    (dict(sigma=1), msadp.MSA_EINVAL),
    (dict(sigma=33), msadp.MSA_EINVAL),
    (dict(packed=1, sigma=5), msadp.MSA_EINVAL),
    (dict(max_len=70000), msadp.MSA_ERANGE),
    (dict(n=-1), msadp.MSA_EINVAL),
    (dict(offsets=None), msadp.MSA_EINVAL),
    (dict(codes=None), msadp.MSA_EINVAL),
])
def test_host_validation_rejects(kw, code):
    L = msadp.lib()
    bad = _seqs(**kw)
    good = _seqs()
    fake = C.c_void_p(16)
    assert L.lev_batch(C.byref(bad), C.byref(good), fake, fake, 4, fake, fake, 1 << 30,
                       None, None) == code
    assert L.nw_batch(C.byref(good), C.byref(bad), fake, fake, 4, fake, fake, fake, fake,
                      1 << 30, None, None) == code
    assert L.lev_allpairs(C.byref(bad), fake, fake, 1 << 30, None, None) == code


def test_host_validation_other_arguments():
    L = msadp.lib()
    g = _seqs()
    fake = C.c_void_p(16)
    # negative pair count, null pair arrays, mismatched alphabets
    assert L.lev_batch(C.byref(g), C.byref(g), fake, fake, -1, fake, fake, 1 << 30, None,
                       None) == msadp.MSA_EINVAL
    assert L.lev_batch(C.byref(g), C.byref(g), None, fake, 4, fake, fake, 1 << 30, None,
                       None) == msadp.MSA_EINVAL
    other = _seqs(sigma=5)
    assert L.lev_batch(C.byref(g), C.byref(other), fake, fake, 4, fake, fake, 1 << 30, None,
                       None) == msadp.MSA_EINVAL
    # zero pairs: success without touching anything
    assert L.lev_batch(C.byref(g), C.byref(g), None, None, 0, None, None, 0, None,
                       None) == msadp.MSA_OK
    assert L.nw_traceback(C.byref(g), C.byref(g), None, None, 0, None, None, None, None, None,
                          None, None) == msadp.MSA_OK
    # workspace too small is reported before any launch
    need = L.lev_workspace_bytes(C.byref(g), C.byref(g), 4)
    assert need > 0
    assert L.lev_batch(C.byref(g), C.byref(g), fake, fake, 4, fake, fake, need - 512, None,
                       None) == msadp.MSA_ENOSPC
    need = L.nw_workspace_bytes(C.byref(g), C.byref(g), 4)
    assert L.nw_batch(C.byref(g), C.byref(g), fake, fake, 4, fake, fake, fake, fake,
                      need - 512, None, None) == msadp.MSA_ENOSPC
    need = L.lev_allpairs_workspace_bytes(C.byref(g))
    assert L.lev_allpairs(C.byref(g), fake, fake, need - 512, None, None) == msadp.MSA_ENOSPC


def test_nw_pattern_length_limit():
    L = msadp.lib()
    a = _seqs(max_len=40000)
    b = _seqs()
    fake = C.c_void_p(16)
    assert L.nw_batch(C.byref(a), C.byref(b), fake, fake, 1, fake, fake, fake, fake, 1 << 40,
                      None, None) == msadp.MSA_ERANGE


def test_probe_host_validation():
    L = msadp.lib()
    fake = C.c_void_p(16)
    ops = C.c_int64(0)
    E = msadp.MSA_EINVAL
    assert L.msa_probe_valu(0, 1, fake, C.byref(ops), None) == E
    assert L.msa_probe_valu(1, 0, fake, C.byref(ops), None) == E
    assert L.msa_probe_valu(1, 1, None, C.byref(ops), None) == E
    assert L.msa_probe_mfma(4, 1, 1, fake, C.byref(ops), None) == E
    assert L.msa_probe_mfma(-1, 1, 1, fake, C.byref(ops), None) == E
    assert L.msa_probe_mfma(0, 1, 1, fake, None, None) == E
    assert L.msa_probe_copy(fake, fake, 24, 1, None) == E            # not a multiple of 16
    assert L.msa_probe_copy(C.c_void_p(8), fake, 32, 1, None) == E   # misaligned
    assert L.msa_probe_copy(fake, fake, 32, 0, None) == E
    assert L.msa_probe_copy(fake, fake, 0, 1, None) == msadp.MSA_OK   # nothing to launch
    assert ops.value == 0


def test_quality_host_validation():
    L = msadp.lib()
    fake = C.c_void_p(256)
    E = msadp.MSA_EINVAL
    assert L.msa_quality_workspace_bytes(4, 10, 64) == 0          # gap code above 63
    assert L.msa_quality_workspace_bytes(-1, 10, 4) == 0
    ws = L.msa_quality_workspace_bytes(4, 10, 4)
    assert ws > 0
    # triangle mode needs rows*(rows-1)/2 pairs; one null pair array is invalid
    assert L.msa_pair_counts(fake, 4, 10, 4, None, None, 5, fake, fake, fake, fake, ws, None,
                             None) == E
    assert L.msa_pair_counts(fake, 4, 10, 4, fake, None, 6, fake, fake, fake, fake, ws, None,
                             None) == E
    assert L.msa_pair_counts(None, 4, 10, 4, None, None, 6, fake, fake, fake, fake, ws, None,
                             None) == E
    assert L.msa_pair_counts(fake, 4, 10, 4, None, None, 6, fake, fake, fake, fake, ws - 512,
                             None, None) == msadp.MSA_ENOSPC
    assert L.msa_pair_counts(fake, 0, 10, 4, fake, fake, 3, fake, fake, fake, fake, ws, None,
                             None) == E                              # pairs but no rows
    # nothing to count: success without a launch
    assert L.msa_pair_counts(fake, 4, 10, 4, fake, fake, 0, None, None, None, None, 0, None,
                             None) == msadp.MSA_OK
    assert L.msa_pair_counts(fake, 1, 10, 4, None, None, 0, None, None, None, None, 0, None,
                             None) == msadp.MSA_OK
    assert L.msa_quality(fake, 4, 10, 70, 10, fake, fake, fake, None, 6, fake, fake, ws, None,
                         None) == E
    assert L.msa_quality(fake, 4, 10, 4, 10, fake, fake, fake, None, 6, None, fake, ws, None,
                         None) == E                                  # no output
    assert L.msa_quality(fake, 4, 10, 4, 10, None, fake, fake, None, 6, fake, fake, ws, None,
                         None) == E
    assert L.msa_quality(fake, 4, 10, 4, 10, fake, fake, fake, None, 6, fake, fake, ws - 512,
                         None, None) == msadp.MSA_ENOSPC
