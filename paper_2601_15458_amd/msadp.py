"""Python face of libmsadp.so: argument marshalling only.

Every computation runs in the HIP library; this module allocates the
caller-owned device buffers (torch tensors), fills the C structs and checks
return codes.  There is no fallback: if the library or a GPU is missing the
calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsadp.so")

MSA_OK, MSA_EINVAL, MSA_ERANGE, MSA_ENOSPC, MSA_EDEVICE = 0, -1, -2, -3, -4
MSA_TUNE_LEV, MSA_TUNE_NW, MSA_TUNE_TREE, MSA_TUNE_PAIRS, MSA_TUNE_TREE_XL = 0, 1, 2, 3, 4
XL_CAP_ALL = (1 << 14) - 1     # an across-lanes cap that takes every cluster


def xl_value(wl: int, sum_cap: int, pole_cap: int) -> int:
    """MSA_TUNE_TREE_XL value: words per lane, and the largest clusters whose
    medoid / pivot / candidate passes (sum_cap) and pole passes (pole_cap)
    run with one pair per group of lanes (include/msadp.h)."""
    return (wl << 28) | (pole_cap << 14) | sum_cap
DS_NAMES = {0: "ok", 1: "symbol code >= sigma", 2: "sequence index out of range",
            3: "length out of range", 4: "output capacity too small",
            5: "non-finite embedding value"}

# Exported entry points and their C signatures (mirrors include/msadp.h).
P = C.c_void_p


class MsaSeqs(C.Structure):
    _fields_ = [("codes", P), ("offsets", P), ("n", C.c_int32), ("sigma", C.c_int32),
                ("max_len", C.c_int32), ("packed_2bit", C.c_int32)]


SP = C.POINTER(MsaSeqs)


class MsaTree(C.Structure):
    _fields_ = [(f, P) for f in ("parent", "left", "right", "center", "lpole", "rpole",
                                 "depth", "mstart", "mcount", "perm")]


TREE_FIELDS = ("parent", "left", "right", "center", "lpole", "rpole", "depth", "mstart",
               "mcount")
SIGNATURES = {
    "msa_strerror": (C.c_char_p, [C.c_int]),
    "msa_version": (C.c_int, []),
    "lev_workspace_bytes": (C.c_size_t, [SP, SP, C.c_int64]),
    "lev_batch": (C.c_int, [SP, SP, P, P, C.c_int64, P, P, C.c_size_t, P, P]),
    "lev_batch_noalloc": (C.c_int, [SP, SP, P, P, C.c_int64, P, P, P]),
    "lev_band_workspace_bytes": (C.c_size_t, [SP, SP, C.c_int64]),
    "lev_band": (C.c_int, [SP, SP, P, P, C.c_int64, C.c_int32, C.c_int32, P, P, P, C.c_size_t,
                           P, P]),
    "lev_allpairs_workspace_bytes": (C.c_size_t, [SP]),
    "lev_allpairs": (C.c_int, [SP, P, P, C.c_size_t, P, P]),
    "nw_tb_bytes": (C.c_size_t, [C.c_int32, C.c_int32]),
    "nw_workspace_bytes": (C.c_size_t, [SP, SP, C.c_int64]),
    "nw_batch": (C.c_int, [SP, SP, P, P, C.c_int64, P, P, P, P, C.c_size_t, P, P]),
    "nw_traceback": (C.c_int, [SP, SP, P, P, C.c_int64, P, P, P, P, P, P, P]),
    "gotoh_tb_bytes": (C.c_size_t, [C.c_int32, C.c_int32]),
    "gotoh_workspace_bytes": (C.c_size_t, [SP, SP, C.c_int64]),
    "gotoh_batch": (C.c_int, [SP, SP, P, P, C.c_int64, P, C.c_int32, C.c_int32, P, P, P, P,
                              C.c_size_t, P, P]),
    "gotoh_traceback": (C.c_int, [SP, SP, P, P, C.c_int64, P, P, P, P, P, P, P]),
    "tree_workspace_bytes": (C.c_size_t, [SP]),
    "tree_build": (C.c_int, [SP, P, C.POINTER(C.c_int32), C.c_int32, P, C.c_size_t, P, P]),
    "tree_build_pruned": (C.c_int, [SP, P, C.c_uint32, C.c_int32, C.c_int32, P,
                                    C.POINTER(C.c_int32), C.c_int32, P, C.c_size_t, P, P]),
    "tree_eval_centers": (C.c_int, [SP, P, C.c_uint32, C.c_int32, C.c_int32, P, C.c_int32, P,
                                    P, P, P, C.c_size_t, P, P]),
    "tree_build_sampled": (C.c_int, [SP, C.c_int32, C.c_int32, C.c_int32, P,
                                     C.POINTER(C.c_int32), C.c_int32, P, C.c_size_t, P, P]),
    "tree_eval_centers_sampled": (C.c_int, [SP, C.c_int32, C.c_int32, C.c_int32, P, C.c_int32,
                                            P, P, P, P, C.c_size_t, P, P]),
    "tree_insert_workspace_bytes": (C.c_size_t, [SP, C.c_int32, C.c_int32]),
    "tree_insert": (C.c_int, [SP, C.c_int32, P, C.c_int32, P, C.POINTER(C.c_int32), P,
                              C.c_size_t, P, P]),
    "msa_merge_workspace_bytes": (C.c_size_t, [SP, C.c_int32, C.c_int32, C.c_size_t]),
    "msa_merge": (C.c_int, [SP, P, C.c_int32, C.c_int32, C.c_size_t, P, C.c_int64,
                            C.POINTER(C.c_int32), P, C.c_size_t, P, P]),
    "msa_tune_set": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "msa_tune_get": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]),
    "msa_tune_clear": (C.c_int, []),
    "msa_tune_candidates": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.c_int32,
                                      C.POINTER(C.c_int32)]),
    "msa_tune_export": (C.c_int, [C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "msa_tune_import": (C.c_int, [C.c_char_p]),
    "msa_autotune_lev": (C.c_int, [SP, P, P, C.c_size_t, C.c_int32, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_float), P, P]),
    "msa_autotune_nw": (C.c_int, [SP, SP, P, P, C.c_int64, P, P, P, P, C.c_size_t, C.c_int32,
                                  C.POINTER(C.c_int32), C.POINTER(C.c_float), P, P]),
    "msa_autotune_pairs": (C.c_int, [SP, SP, P, P, C.c_int64, P, P, C.c_size_t, C.c_int32,
                                     C.POINTER(C.c_int32), C.POINTER(C.c_float), P, P]),
    "msa_autotune_tree": (C.c_int, [SP, P, C.POINTER(C.c_int32), C.c_int32, P, C.c_size_t,
                                    C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_float), P, P]),
    "msa_autotune_tree_xl": (C.c_int, [SP, C.c_int32, C.c_int32, P, C.POINTER(C.c_int32),
                                       C.c_int32, P, C.c_size_t, C.c_int32,
                                       C.POINTER(C.c_int32), C.POINTER(C.c_float), P, P]),
    "cnn_param_bytes": (C.c_size_t, []),
    "cnn_set_params": (C.c_int, [P, P, P, P]),
    "cnn_get_params": (C.c_int, [P, P, P, P, P, P]),
    "cnn_workspace_bytes": (C.c_size_t, [SP, C.c_int32, C.c_int64, C.c_int32]),
    "cnn_embed": (C.c_int, [P, SP, P, C.c_int32, C.c_int64, P, P, C.c_size_t, P, P]),
    "cnn_train_step": (C.c_int, [P, SP, P, C.c_int32, C.c_int64, P, P, P, C.c_int32, C.c_float,
                                 C.c_int32, P, P, C.c_size_t, P, P]),
    "msa_quality_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32]),
    "msa_pair_counts": (C.c_int, [P, C.c_int32, C.c_int32, C.c_int32, P, P, C.c_int64, P, P, P,
                                  P, C.c_size_t, P, P]),
    "msa_quality": (C.c_int, [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P, P, P,
                              C.c_int64, P, P, C.c_size_t, P, P]),
    "msa_probe_valu": (C.c_int, [C.c_int32, C.c_int32, P, C.POINTER(C.c_int64), P]),
    "msa_probe_mfma": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, P, C.POINTER(C.c_int64), P]),
    "msa_probe_copy": (C.c_int, [P, P, C.c_size_t, C.c_int32, P]),
}

_lib = None


def lib():
    """Load libmsadp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class MsaError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {lib().msa_strerror(code).decode()} ({code})")


def _check(rc: int, where: str):
    if rc != MSA_OK:
        raise MsaError(rc, where)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _device():
    if not torch.cuda.is_available():
        raise RuntimeError("msadp needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch.device("cuda", torch.cuda.current_device())


@dataclass
class Seqs:
    """A sequence set resident on the GPU in CSR form (see include/msadp.h)."""
    codes: torch.Tensor       # uint8 on the device
    offsets: torch.Tensor     # int64 [n+1] on the device
    lengths: np.ndarray       # host copy of the n lengths (for output sizing)
    sigma: int
    max_len: int
    packed_2bit: bool = False

    @property
    def n(self) -> int:
        return len(self.lengths)

    def struct(self) -> MsaSeqs:
        return MsaSeqs(self.codes.data_ptr() if self.codes.numel() else None,
                       self.offsets.data_ptr(), self.n, self.sigma, self.max_len,
                       int(self.packed_2bit))


def to_device(codes, offsets, sigma, max_len=None, packed_2bit=False, device=None) -> Seqs:
    """Copy a host CSR set to the GPU.  With packed_2bit, `codes` must already
    hold four 2-bit symbols per byte (symbol p in bits 2*(p%4) of byte p//4)."""
    dev = device or _device()
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    lengths = np.diff(offsets)
    if max_len is None:
        max_len = int(lengths.max()) if len(lengths) else 0
    c = torch.from_numpy(np.ascontiguousarray(codes, dtype=np.uint8)).to(dev)
    if c.numel() == 0:
        c = torch.zeros(16, dtype=torch.uint8, device=dev)
    o = torch.from_numpy(offsets).to(dev)
    return Seqs(c, o, lengths, int(sigma), int(max_len), bool(packed_2bit))


def pack_2bit_host(codes) -> np.ndarray:
    """Host-side packing for building test inputs (four symbols per byte)."""
    c = np.asarray(codes, dtype=np.uint8)
    pad = (-len(c)) % 4
    c = np.concatenate([c, np.zeros(pad, np.uint8)]).reshape(-1, 4)
    return (c[:, 0] | (c[:, 1] << 2) | (c[:, 2] << 4) | (c[:, 3] << 6)).astype(np.uint8)


def _i32(x, dev):
    if isinstance(x, torch.Tensor):
        return x.to(device=dev, dtype=torch.int32).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.int32), device=dev)


class Status:
    """Device status word (first device-detected error wins)."""

    def __init__(self, dev):
        self.t = torch.zeros(1, dtype=torch.int32, device=dev)

    def check(self, where):
        v = int(self.t.item())
        if v != 0:
            raise RuntimeError(f"{where}: device reported {DS_NAMES.get(v, v)}")


class LevBatch:
    """Reusable lev_batch launcher: pairs on the device, workspace sized once."""

    def __init__(self, A: Seqs, B: Seqs, ia, ib, out=None):
        dev = A.codes.device
        self.A, self.B = A, B
        self.ia, self.ib = _i32(ia, dev), _i32(ib, dev)
        self.n_pairs = self.ia.numel()
        if out is None:
            out = torch.empty(max(self.n_pairs, 1), dtype=torch.uint16, device=dev)
        self.out = out
        self.sa, self.sb = A.struct(), B.struct()
        self.wsb = lib().lev_workspace_bytes(C.byref(self.sa), C.byref(self.sb), self.n_pairs)
        self.ws = torch.empty(max(self.wsb, 1), dtype=torch.uint8, device=dev)
        self.st = Status(dev)

    def args(self):
        """lev_batch's arguments up to the workspace size."""
        return (C.byref(self.sa), C.byref(self.sb), _ptr(self.ia), _ptr(self.ib), self.n_pairs,
                _ptr(self.out), _ptr(self.ws), self.wsb)

    def __call__(self, stream=None):
        rc = lib().lev_batch(*self.args(), _ptr(self.st.t), _stream(stream))
        _check(rc, "lev_batch")
        return self.out[: self.n_pairs]


def lev_batch(A: Seqs, B: Seqs, ia, ib, out=None, stream=None, check=True):
    """uint16 distances lev(A[ia[p]], B[ib[p]])."""
    lb = LevBatch(A, B, ia, ib, out)
    res = lb(stream)
    if check:
        lb.st.check("lev_batch")
    return res


BAND_NONE = 0xFFFF


class LevBand:
    """Reusable exact banded Levenshtein launcher (lev_band): distances up to
    kmax, 0xFFFF beyond; k_used holds the band threshold that verified each."""

    def __init__(self, A: Seqs, B: Seqs, ia, ib, k0: int = 256, kmax: int = 4000):
        dev = A.codes.device
        self.A, self.B = A, B
        self.ia, self.ib = _i32(ia, dev), _i32(ib, dev)
        self.n_pairs = self.ia.numel()
        self.k0, self.kmax = int(k0), int(kmax)
        self.out = torch.empty(max(self.n_pairs, 1), dtype=torch.uint16, device=dev)
        self.k_used = torch.empty(max(self.n_pairs, 1), dtype=torch.int32, device=dev)
        self.sa, self.sb = A.struct(), B.struct()
        self.wsb = lib().lev_band_workspace_bytes(C.byref(self.sa), C.byref(self.sb),
                                                  self.n_pairs)
        self.ws = torch.empty(max(self.wsb, 1), dtype=torch.uint8, device=dev)
        self.st = Status(dev)

    def __call__(self, stream=None):
        rc = lib().lev_band(C.byref(self.sa), C.byref(self.sb), _ptr(self.ia), _ptr(self.ib),
                            self.n_pairs, self.k0, self.kmax, _ptr(self.out), _ptr(self.k_used),
                            _ptr(self.ws), self.wsb, _ptr(self.st.t), _stream(stream))
        _check(rc, "lev_band")
        return self.out[: self.n_pairs]


def lev_band(A: Seqs, B: Seqs, ia, ib, k0: int = 256, kmax: int = 4000, stream=None):
    """(distances uint16 (0xFFFF above kmax), verifying thresholds int32)."""
    lb = LevBand(A, B, ia, ib, k0, kmax)
    d = lb(stream)
    lb.st.check("lev_band")
    return d, lb.k_used[: lb.n_pairs]


NOALLOC_SCRATCH_BYTES = 64 << 20


def lev_batch_noalloc(A: Seqs, B: Seqs, ia, ib, out=None, stream=None, check=True):
    """lev_batch with the library's fixed device workspace (no workspace
    buffer is allocated here; inputs and the output are the caller's)."""
    dev = A.codes.device
    ia, ib = _i32(ia, dev), _i32(ib, dev)
    n_pairs = ia.numel()
    if out is None:
        out = torch.empty(max(n_pairs, 1), dtype=torch.uint16, device=dev)
    sa, sb = A.struct(), B.struct()
    st = Status(dev)
    rc = lib().lev_batch_noalloc(C.byref(sa), C.byref(sb), _ptr(ia), _ptr(ib), n_pairs,
                                 _ptr(out), _ptr(st.t), _stream(stream))
    _check(rc, "lev_batch_noalloc")
    if check:
        st.check("lev_batch_noalloc")
    return out[:n_pairs]


class AllPairs:
    """Reusable all-pairs launcher: workspace sized once, output preallocated."""

    def __init__(self, A: Seqs):
        self.A = A
        dev = A.codes.device
        self.sa = A.struct()
        n = A.n
        self.out = torch.empty(max(n * (n - 1) // 2, 1), dtype=torch.uint16, device=dev)
        self.wsb = lib().lev_allpairs_workspace_bytes(C.byref(self.sa))
        self.ws = torch.empty(max(self.wsb, 1), dtype=torch.uint8, device=dev)
        self.st = Status(dev)

    def __call__(self, stream=None):
        rc = lib().lev_allpairs(C.byref(self.sa), _ptr(self.out), _ptr(self.ws), self.wsb,
                                _ptr(self.st.t), _stream(stream))
        _check(rc, "lev_allpairs")
        return self.out


def lev_allpairs(A: Seqs, stream=None):
    """Condensed uint16 distances of every pair i < j of A."""
    ap = AllPairs(A)
    out = ap(stream)
    ap.st.check("lev_allpairs")
    n = A.n
    return out[: n * (n - 1) // 2]


class NwResult:
    def __init__(self, score, tb, tb_offsets, n_pairs):
        self.score, self.tb, self.tb_offsets, self.n_pairs = score, tb, tb_offsets, n_pairs


class NwBatch:
    """Reusable NW launcher: buffers sized once for fixed (A, B, ia, ib)."""

    def __init__(self, A: Seqs, B: Seqs, ia, ib):
        self.A, self.B = A, B
        self.r = nw_batch(A, B, ia, ib)
        r = self.r
        dev = A.codes.device
        self.sa, self.sb = A.struct(), B.struct()
        self.wsb = lib().nw_workspace_bytes(C.byref(self.sa), C.byref(self.sb), r.n_pairs)
        self.ws = torch.empty(max(self.wsb, 1), dtype=torch.uint8, device=dev)
        caps = (r.m + r.n).astype(np.int64)
        self.ops_off = np.zeros(r.n_pairs + 1, dtype=np.int64)
        np.cumsum(caps, out=self.ops_off[1:])
        self.ops = torch.empty(max(int(self.ops_off[-1]), 1), dtype=torch.uint8, device=dev)
        self.ops_off_d = torch.from_numpy(self.ops_off).to(dev)
        self.ops_len = torch.empty(max(r.n_pairs, 1), dtype=torch.int32, device=dev)
        self.st = Status(dev)

    def fill_args(self):
        """nw_batch's arguments up to the workspace size."""
        r = self.r
        return (C.byref(self.sa), C.byref(self.sb), _ptr(r.ia), _ptr(r.ib), r.n_pairs,
                _ptr(r.score), _ptr(r.tb), _ptr(r.tb_offsets), _ptr(self.ws), self.wsb)

    def fill(self, stream=None):
        rc = lib().nw_batch(*self.fill_args(), _ptr(self.st.t), _stream(stream))
        _check(rc, "nw_batch")

    def traceback(self, stream=None):
        r = self.r
        rc = lib().nw_traceback(C.byref(self.sa), C.byref(self.sb), _ptr(r.ia), _ptr(r.ib),
                                r.n_pairs, _ptr(r.tb), _ptr(r.tb_offsets), _ptr(self.ops),
                                _ptr(self.ops_off_d), _ptr(self.ops_len), _ptr(self.st.t),
                                _stream(stream))
        _check(rc, "nw_traceback")


def nw_batch(A: Seqs, B: Seqs, ia, ib, stream=None, check=True) -> NwResult:
    """Fill: int32 scores and the traceback codes of every pair."""
    dev = A.codes.device
    ia_h = np.ascontiguousarray(ia.cpu().numpy() if isinstance(ia, torch.Tensor) else ia,
                                dtype=np.int32)
    ib_h = np.ascontiguousarray(ib.cpu().numpy() if isinstance(ib, torch.Tensor) else ib,
                                dtype=np.int32)
    n_pairs = len(ia_h)
    m = A.lengths[ia_h] if n_pairs else np.zeros(0, np.int64)
    n = B.lengths[ib_h] if n_pairs else np.zeros(0, np.int64)
    sizes = np.array([lib().nw_tb_bytes(int(a), int(b)) for a, b in zip(m, n)], dtype=np.int64)
    sizes = (sizes + 255) // 256 * 256
    tb_off = np.zeros(n_pairs + 1, dtype=np.int64)
    np.cumsum(sizes, out=tb_off[1:])
    tb = torch.empty(max(int(tb_off[-1]), 256), dtype=torch.uint8, device=dev)
    tb_off_d = torch.from_numpy(tb_off).to(dev)
    score = torch.empty(max(n_pairs, 1), dtype=torch.int32, device=dev)
    ia_d, ib_d = _i32(ia_h, dev), _i32(ib_h, dev)
    sa, sb = A.struct(), B.struct()
    wsb = lib().nw_workspace_bytes(C.byref(sa), C.byref(sb), n_pairs)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    st = Status(dev)
    rc = lib().nw_batch(C.byref(sa), C.byref(sb), _ptr(ia_d), _ptr(ib_d), n_pairs, _ptr(score),
                        _ptr(tb), _ptr(tb_off_d), _ptr(ws), wsb, _ptr(st.t), _stream(stream))
    _check(rc, "nw_batch")
    if check:
        st.check("nw_batch")
    r = NwResult(score[:n_pairs], tb, tb_off_d, n_pairs)
    r.ia, r.ib, r.m, r.n = ia_d, ib_d, m, n
    return r


def nw_traceback(A: Seqs, B: Seqs, r: NwResult, stream=None, check=True):
    """Alignments (list of uint8 op arrays, 0=M 1=D 2=I) for a nw_batch result."""
    dev = A.codes.device
    caps = (r.m + r.n).astype(np.int64)
    ops_off = np.zeros(r.n_pairs + 1, dtype=np.int64)
    np.cumsum(caps, out=ops_off[1:])
    ops = torch.empty(max(int(ops_off[-1]), 1), dtype=torch.uint8, device=dev)
    ops_off_d = torch.from_numpy(ops_off).to(dev)
    ops_len = torch.empty(max(r.n_pairs, 1), dtype=torch.int32, device=dev)
    sa, sb = A.struct(), B.struct()
    st = Status(dev)
    rc = lib().nw_traceback(C.byref(sa), C.byref(sb), _ptr(r.ia), _ptr(r.ib), r.n_pairs,
                            _ptr(r.tb), _ptr(r.tb_offsets), _ptr(ops), _ptr(ops_off_d),
                            _ptr(ops_len), _ptr(st.t), _stream(stream))
    _check(rc, "nw_traceback")
    if check:
        st.check("nw_traceback")
    return ops, ops_off, ops_len[: r.n_pairs]


class GotohBatch:
    """Affine-gap NW (substitution matrix `sub`, sigma x sigma, a gap run of
    k scoring -(open + k ext)) over fixed pairs: buffers sized once; fill()
    computes scores and traceback codes, traceback() the alignments."""

    def __init__(self, A: Seqs, B: Seqs, ia, ib, sub, open_: int, ext: int):
        dev = A.codes.device
        self.A, self.B = A, B
        self.ia_h = np.ascontiguousarray(ia.cpu().numpy() if isinstance(ia, torch.Tensor) else ia,
                                         dtype=np.int32)
        self.ib_h = np.ascontiguousarray(ib.cpu().numpy() if isinstance(ib, torch.Tensor) else ib,
                                         dtype=np.int32)
        self.n_pairs = P_ = len(self.ia_h)
        self.sub = np.ascontiguousarray(sub, dtype=np.int32)
        self.open, self.ext = int(open_), int(ext)
        # sizes only: an index out of range is reported by the device
        self.m = A.lengths[np.clip(self.ia_h, 0, max(A.n - 1, 0))] if P_ else np.zeros(0, np.int64)
        self.n = B.lengths[np.clip(self.ib_h, 0, max(B.n - 1, 0))] if P_ else np.zeros(0, np.int64)
        sizes = np.array([lib().gotoh_tb_bytes(int(a), int(b)) for a, b in zip(self.m, self.n)],
                         dtype=np.int64)
        sizes = (sizes + 255) // 256 * 256
        tb_off = np.zeros(P_ + 1, dtype=np.int64)
        np.cumsum(sizes, out=tb_off[1:])
        self.tb = torch.empty(max(int(tb_off[-1]), 256), dtype=torch.uint8, device=dev)
        self.tb_off = torch.from_numpy(tb_off).to(dev)
        self.score = torch.empty(max(P_, 1), dtype=torch.int32, device=dev)
        self.ia, self.ib = _i32(self.ia_h, dev), _i32(self.ib_h, dev)
        self.sa, self.sb = A.struct(), B.struct()
        self.wsb = lib().gotoh_workspace_bytes(C.byref(self.sa), C.byref(self.sb), P_)
        self.ws = torch.empty(max(self.wsb, 1), dtype=torch.uint8, device=dev)
        caps = (self.m + self.n).astype(np.int64)
        self.ops_off = np.zeros(P_ + 1, dtype=np.int64)
        np.cumsum(caps, out=self.ops_off[1:])
        self.ops = torch.empty(max(int(self.ops_off[-1]), 1), dtype=torch.uint8, device=dev)
        self.ops_off_d = torch.from_numpy(self.ops_off).to(dev)
        self.ops_len = torch.empty(max(P_, 1), dtype=torch.int32, device=dev)
        self.st = Status(dev)

    def fill(self, stream=None):
        rc = lib().gotoh_batch(C.byref(self.sa), C.byref(self.sb), _ptr(self.ia), _ptr(self.ib),
                               self.n_pairs, self.sub.ctypes.data_as(C.c_void_p), self.open,
                               self.ext, _ptr(self.score), _ptr(self.tb), _ptr(self.tb_off),
                               _ptr(self.ws), self.wsb, _ptr(self.st.t), _stream(stream))
        _check(rc, "gotoh_batch")
        return self.score[: self.n_pairs]

    def traceback(self, stream=None):
        rc = lib().gotoh_traceback(C.byref(self.sa), C.byref(self.sb), _ptr(self.ia),
                                   _ptr(self.ib), self.n_pairs, _ptr(self.tb), _ptr(self.tb_off),
                                   _ptr(self.ops), _ptr(self.ops_off_d), _ptr(self.ops_len),
                                   _ptr(self.st.t), _stream(stream))
        _check(rc, "gotoh_traceback")

    def results(self):
        """(scores int64[P], list of op arrays) on the host."""
        self.st.check("gotoh")
        sc = self.score[: self.n_pairs].cpu().numpy().astype(np.int64)
        return sc, split_ops(self.ops, self.ops_off, self.ops_len[: self.n_pairs])


def gotoh(A: Seqs, B: Seqs, ia, ib, sub, open_: int, ext: int, stream=None):
    """Scores and alignments of affine-gap NW over the pairs (host arrays)."""
    g = GotohBatch(A, B, ia, ib, sub, open_, ext)
    g.fill(stream)
    g.traceback(stream)
    return g.results()


def split_ops(ops, ops_off, ops_len):
    """Host list of per-pair op arrays."""
    o = ops.cpu().numpy()
    L = ops_len.cpu().numpy()
    return [o[ops_off[p]: ops_off[p] + L[p]].copy() for p in range(len(L))]


class Tree:
    """Device arrays of a guide tree (capacity 2n - 1 nodes)."""

    def __init__(self, n, dev):
        cap = max(2 * n - 1, 1)
        self.t = {f: torch.full((cap,), -1, dtype=torch.int64 if f in ("mstart", "mcount")
                                else torch.int32, device=dev) for f in TREE_FIELDS}
        self.t["perm"] = torch.zeros(max(n, 1), dtype=torch.int32, device=dev)
        self.n_nodes = 0
        self.n = n

    def struct(self):
        return MsaTree(*[self.t[f].data_ptr() for f in TREE_FIELDS + ("perm",)])

    @classmethod
    def from_host(cls, h, dev):
        """Device copy of a host tree dict (as returned by tree_build)."""
        n = len(h["perm"])
        t = cls(n, dev)
        k = int(h["n_nodes"])
        for f in TREE_FIELDS:
            t.t[f][:k] = torch.as_tensor(np.asarray(h[f][:k]), dtype=t.t[f].dtype).to(dev)
        t.t["perm"][:n] = torch.as_tensor(np.asarray(h["perm"]), dtype=torch.int32).to(dev)
        t.n_nodes = k
        return t

    def host(self):
        k = self.n_nodes
        out = {f: self.t[f][:k].cpu().numpy() for f in TREE_FIELDS}
        out["perm"] = self.t["perm"][: self.n].cpu().numpy()
        out["n_nodes"] = k
        return out


class TreeBuilder:
    """Reusable Alg. 1 builder for one sequence set.  With emb (device
    float32 [n, 128]) the medoid is pruned to the topk members that the
    embedding ranks first (tree_build_pruned); emb_offset is the calibration
    offset added to every embedding distance.  With pivots > 0 (and no emb)
    the topk members closest in sum to `pivots` hashed members are the
    candidates (tree_build_sampled)."""

    def __init__(self, S: Seqs, use_graph=False, emb=None, topk=16, exact_below=0,
                 emb_offset=0.0, pivots=0):
        self.S = S
        self.pivots = int(pivots)
        if self.pivots and emb is not None:
            raise ValueError("pivots and emb select different rankings: give one")
        if emb is not None:
            if (emb.dtype != torch.float32 or emb.device != S.codes.device
                    or tuple(emb.shape) != (S.n, 128) or not emb.is_contiguous()):
                raise ValueError("emb must be a contiguous float32 [n, 128] tensor on the device")
        self.emb = emb
        self.topk = int(topk)
        self.exact_below = int(exact_below)
        self.emb_q0 = emb_offset_q(emb_offset)
        dev = S.codes.device
        self.ss = S.struct()
        self.tree = Tree(S.n, dev)
        self.ts = self.tree.struct()
        self.wsb = lib().tree_workspace_bytes(C.byref(self.ss))
        self.ws = torch.empty(max(self.wsb, 1), dtype=torch.uint8, device=dev)
        self.st = Status(dev)
        self.use_graph = bool(use_graph)

    def __call__(self, stream=None):
        nn = C.c_int32(0)
        if self.pivots:
            rc = lib().tree_build_sampled(C.byref(self.ss), self.pivots, self.topk,
                                          self.exact_below, C.byref(self.ts), C.byref(nn),
                                          int(self.use_graph), _ptr(self.ws), self.wsb,
                                          _ptr(self.st.t), _stream(stream))
            _check(rc, "tree_build_sampled")
        elif self.emb is None:
            rc = lib().tree_build(C.byref(self.ss), C.byref(self.ts), C.byref(nn),
                                  int(self.use_graph), _ptr(self.ws), self.wsb, _ptr(self.st.t),
                                  _stream(stream))
            _check(rc, "tree_build")
        else:
            rc = lib().tree_build_pruned(C.byref(self.ss), _ptr(self.emb), self.emb_q0, self.topk,
                                         self.exact_below, C.byref(self.ts), C.byref(nn),
                                         int(self.use_graph),
                                         _ptr(self.ws), self.wsb, _ptr(self.st.t), _stream(stream))
            _check(rc, "tree_build_pruned")
        self.tree.n_nodes = nn.value
        return self.tree


def emb_offset_q(offset: float) -> int:
    """A calibration offset in the library's fixed point (units of 2^-16)."""
    q = int(round(float(offset) * 65536.0))
    if not 0 <= q <= 1 << 31:
        raise ValueError("emb_offset must lie in [0, 2^15]")
    return q


def tree_build(S: Seqs, use_graph=False, stream=None, emb=None, topk=16, exact_below=0,
               emb_offset=0.0, pivots=0):
    """Alg. 1 guide tree of S; returns host numpy arrays like the oracle's.
    emb/topk/exact_below/emb_offset select the surrogate-pruned medoid,
    pivots/topk/exact_below the sampled one (see TreeBuilder)."""
    if use_graph and stream is None:
        stream = torch.cuda.Stream()
    tb = TreeBuilder(S, use_graph, emb, topk, exact_below, emb_offset, pivots)
    with torch.cuda.stream(stream) if stream is not None else _nullctx():
        t = tb(stream)
    torch.cuda.synchronize()
    tb.st.check("tree_build")
    return t.host()


def tree_insert(S: Seqs, n_old: int, tree, stream=None) -> Tree:
    """Online insertion: S holds the n_old sequences `tree` (a device Tree or
    a host dict from tree_build) was built on, followed by new ones.  Each
    new sequence is routed down by the poles' split rule, the leaves that
    receive some are re-partitioned by Alg. 1, and the tree is renumbered
    breadth-first (tree_insert in the library).  Returns a device Tree over
    all of S; msa_merge(S, tree) aligns the grown set."""
    dev = S.codes.device
    if isinstance(tree, dict):
        tree = Tree.from_host(tree, dev)
    out = Tree(S.n, dev)
    ss, to, tn = S.struct(), tree.struct(), out.struct()
    wsb = lib().tree_insert_workspace_bytes(C.byref(ss), int(n_old), tree.n_nodes)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    st = Status(dev)
    nn = C.c_int32(0)
    rc = lib().tree_insert(C.byref(ss), int(n_old), C.byref(to), tree.n_nodes, C.byref(tn),
                           C.byref(nn), _ptr(ws), wsb, _ptr(st.t), _stream(stream))
    _check(rc, "tree_insert")
    torch.cuda.synchronize()
    st.check("tree_insert")
    out.n_nodes = nn.value
    return out


def tree_eval_centers(S: Seqs, tree, emb=None, topk=16, exact_below=0, emb_offset=0.0,
                      stream=None, pivots=0):
    """(center, lpole, rpole) host arrays that the build picks for each node
    of `tree` (a device Tree) when that node's members are given: the full
    median (emb None, pivots 0), the embedding-pruned one, or the sampled
    one (pivots > 0)."""
    dev = S.codes.device
    if isinstance(tree, dict):
        tree = Tree.from_host(tree, dev)
    if emb is not None and (emb.dtype != torch.float32 or tuple(emb.shape) != (S.n, 128)
                            or not emb.is_contiguous() or emb.device != dev):
        raise ValueError("emb must be a contiguous float32 [n, 128] tensor on the device")
    nn = tree.n_nodes
    out = [torch.full((max(nn, 1),), -1, dtype=torch.int32, device=dev) for _ in range(3)]
    ss, ts = S.struct(), tree.struct()
    wsb = lib().tree_workspace_bytes(C.byref(ss))
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    st = Status(dev)
    if pivots:
        if emb is not None:
            raise ValueError("pivots and emb select different rankings: give one")
        rc = lib().tree_eval_centers_sampled(C.byref(ss), int(pivots), int(topk),
                                             int(exact_below), C.byref(ts), nn,
                                             *[_ptr(o) for o in out], _ptr(ws), wsb,
                                             _ptr(st.t), _stream(stream))
    else:
        rc = lib().tree_eval_centers(C.byref(ss), _ptr(emb), emb_offset_q(emb_offset), int(topk),
                                     int(exact_below),
                                     C.byref(ts), nn,
                                     *[_ptr(o) for o in out], _ptr(ws), wsb, _ptr(st.t),
                                     _stream(stream))
    _check(rc, "tree_eval_centers")
    torch.cuda.synchronize()
    st.check("tree_eval_centers")
    return tuple(o[:nn].cpu().numpy() for o in out)


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


def msa_merge(S: Seqs, tree: Tree, width_cap=None, tb_cap=1 << 30, stream=None):
    """Final alignment (host uint8 array n x W, gap code = sigma) of S along
    a tree built on the device.  width_cap grows until the alignment fits."""
    dev = S.codes.device
    cap = width_cap or min(32768, max(64, 2 * S.max_len))
    ss, ts = S.struct(), tree.struct()
    while True:
        pitch = (cap + 15) // 16 * 16
        out = torch.empty(max(S.n * pitch, 1), dtype=torch.uint8, device=dev)
        wsb = lib().msa_merge_workspace_bytes(C.byref(ss), tree.n_nodes, cap, tb_cap)
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
        st = Status(dev)
        w = C.c_int32(0)
        rc = lib().msa_merge(C.byref(ss), C.byref(ts), tree.n_nodes, cap, tb_cap, _ptr(out),
                             pitch, C.byref(w), _ptr(ws), wsb, _ptr(st.t), _stream(stream))
        if rc == MSA_ENOSPC and width_cap is None and (cap < 32768 or tb_cap < (1 << 36)):
            # the width or one level's traceback codes did not fit: grow both
            cap = min(32768, cap * 2)
            tb_cap = min(1 << 36, tb_cap * 2)
            continue
        _check(rc, "msa_merge")
        torch.cuda.synchronize()
        st.check("msa_merge")
        W = w.value
        return out[: S.n * pitch].view(S.n, pitch)[:, :W].cpu().numpy()


def align(S: Seqs, use_graph=False, stream=None):
    """Guide tree (Alg. 1) then the bottom-up merge: (tree dict, alignment)."""
    tb = TreeBuilder(S, use_graph)
    if use_graph and stream is None:
        stream = torch.cuda.Stream()
    with torch.cuda.stream(stream) if stream is not None else _nullctx():
        tree = tb(stream)
        torch.cuda.synchronize()
        tb.st.check("tree_build")
        msa = msa_merge(S, tree, stream=stream)
    return tree.host(), msa


# ------------------------------------------------------- alignment quality
QUALITY_FIELDS = ("pct_gaps", "p_min", "p_avg", "p_max", "distortion", "stretch",
                  "n_p_pairs", "n_d_pairs")


def _msa_dev(msa):
    if isinstance(msa, torch.Tensor):
        return msa.to(device=_device(), dtype=torch.uint8).contiguous()
    return torch.from_numpy(np.ascontiguousarray(msa, dtype=np.uint8)).to(_device())


class Quality:
    """Alignment-quality metrics (msa_pair_counts, msa_quality) of one
    alignment held on the device: rows x width codes, `gap` the gap code."""

    def __init__(self, msa, gap: int):
        self.msa = _msa_dev(msa)
        self.rows, self.width = (int(x) for x in self.msa.shape)
        self.gap = int(gap)
        self.wsb = lib().msa_quality_workspace_bytes(self.rows, self.width, self.gap)
        if self.wsb == 0:
            raise MsaError(MSA_EINVAL, "msa_quality_workspace_bytes")
        self.ws = torch.empty(self.wsb, dtype=torch.uint8, device=self.msa.device)
        self.st = Status(self.msa.device)

    def pair_counts(self, ia=None, ib=None, stream=None):
        """(hamming, aligned, mismatched) int32 device tensors; all pairs
        i < j in condensed order when ia and ib are None."""
        dev = self.msa.device
        if ia is None:
            n = self.rows * (self.rows - 1) // 2
            dia = dib = None
        else:
            dia, dib = _i32(ia, dev), _i32(ib, dev)
            n = int(dia.numel())
        h = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        al = torch.empty_like(h)
        mm = torch.empty_like(h)
        rc = lib().msa_pair_counts(_ptr(self.msa), self.rows, self.width, self.gap, _ptr(dia),
                                   _ptr(dib), n, _ptr(h), _ptr(al), _ptr(mm), _ptr(self.ws),
                                   self.wsb, _ptr(self.st.t), _stream(stream))
        _check(rc, "msa_pair_counts")
        return h[:n], al[:n], mm[:n]

    def metrics(self, counts, max_len: int, lev=None, stream=None):
        """Dict of QUALITY_FIELDS from pair_counts' output and the pairs'
        Levenshtein distances (device uint16 tensor, same order) or None."""
        h, al, mm = counts
        n = int(h.numel())
        for t in (h, al, mm):
            assert t.dtype == torch.int32 and t.is_cuda and t.numel() == n and t.is_contiguous()
        if lev is not None:
            assert lev.dtype == torch.uint16 and lev.is_cuda and lev.is_contiguous()
            assert lev.numel() >= n, "one distance per pair"
        out = torch.zeros(8, dtype=torch.float64, device=self.msa.device)
        rc = lib().msa_quality(_ptr(self.msa), self.rows, self.width, self.gap, int(max_len),
                               _ptr(h), _ptr(al), _ptr(mm), _ptr(lev), n, _ptr(out),
                               _ptr(self.ws), self.wsb, _ptr(self.st.t), _stream(stream))
        _check(rc, "msa_quality")
        v = out.cpu().numpy()
        self.st.check("msa_quality")
        d = dict(zip(QUALITY_FIELDS, (float(x) for x in v)))
        d["n_p_pairs"], d["n_d_pairs"] = int(v[6]), int(v[7])
        return d


# ---------------------------------------------------------------- tuning
def tune_set(kind: int, sigma: int, bin_: int, value: int):
    _check(lib().msa_tune_set(kind, sigma, bin_, value), "msa_tune_set")


def tune_get(kind: int, sigma: int, bin_: int) -> int:
    """The table's value for the key, 0 when it holds none."""
    v = C.c_int32(0)
    _check(lib().msa_tune_get(kind, sigma, bin_, C.byref(v)), "msa_tune_get")
    return v.value


def tune_clear():
    _check(lib().msa_tune_clear(), "msa_tune_clear")


def tune_candidates(kind: int):
    vals = (C.c_int32 * 16)()
    n = C.c_int32(0)
    _check(lib().msa_tune_candidates(kind, vals, 16, C.byref(n)), "msa_tune_candidates")
    return [vals[i] for i in range(n.value)]


def tune_export() -> str:
    n = C.c_size_t(0)
    rc = lib().msa_tune_export(None, 0, C.byref(n))
    if rc not in (MSA_OK, MSA_ENOSPC):
        _check(rc, "msa_tune_export")
    buf = C.create_string_buffer(n.value + 1)
    _check(lib().msa_tune_export(buf, n.value + 1, C.byref(n)), "msa_tune_export")
    return buf.value.decode()


def tune_import(text: str):
    _check(lib().msa_tune_import(text.encode()), "msa_tune_import")


def tune_save(path: str):
    """Write the tuning table to a JSON cache file."""
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    with open(path, "w") as f:
        f.write(tune_export() + "\n")


def tune_load(path: str) -> bool:
    """Merge a JSON cache file into the table (False if it does not exist)."""
    if not os.path.exists(path):
        return False
    with open(path) as f:
        tune_import(f.read())
    return True


def lev_words_bin(S: Seqs) -> int:
    return max(1, (S.max_len + 63) // 64)


def autotune_lev(S: Seqs, reps: int = 2, stream=None):
    """Time the lev_allpairs variants on S and keep the fastest in the table;
    returns (words per pass, ms per call)."""
    ap = AllPairs(S)
    best, ms = C.c_int32(0), C.c_float(0.0)
    rc = lib().msa_autotune_lev(C.byref(ap.sa), _ptr(ap.out), _ptr(ap.ws), ap.wsb, int(reps),
                                C.byref(best), C.byref(ms), _ptr(ap.st.t), _stream(stream))
    _check(rc, "msa_autotune_lev")
    ap.st.check("msa_autotune_lev")
    return best.value, ms.value


def autotune_pairs(lb: "LevBatch", reps: int = 2, stream=None):
    """Time the lev_batch pair layouts on a prepared LevBatch and keep the
    fastest; returns (the layout: 1 one pair per lane, 2 a pair per group
    of lanes, 64 pairs grouped by pattern; ms per call)."""
    best, ms = C.c_int32(0), C.c_float(0.0)
    rc = lib().msa_autotune_pairs(*lb.args(), int(reps), C.byref(best), C.byref(ms),
                                  _ptr(lb.st.t), _stream(stream))
    _check(rc, "msa_autotune_pairs")
    lb.st.check("msa_autotune_pairs")
    return best.value, ms.value


def pairs_words_bin(A: Seqs, B: Seqs) -> int:
    """Tuning-table bin of a lev_batch call (MSA_TUNE_PAIRS)."""
    return max(1, (max(A.max_len, B.max_len) + 63) // 64)


def autotune_nw(nb: "NwBatch", reps: int = 2, stream=None):
    """Time the nw_batch variants on a prepared NwBatch and keep the fastest;
    returns (steps between barriers, ms per call)."""
    best, ms = C.c_int32(0), C.c_float(0.0)
    rc = lib().msa_autotune_nw(*nb.fill_args(), int(reps), C.byref(best), C.byref(ms),
                               _ptr(nb.st.t), _stream(stream))
    _check(rc, "msa_autotune_nw")
    nb.st.check("msa_autotune_nw")
    return best.value, ms.value


def autotune_tree(S: Seqs, reps: int = 1, use_graph=True, stream=None):
    """Time the exact tree build per kernel class on S and keep the fastest
    in the table; returns (words per pass, ms per build)."""
    if use_graph and stream is None:
        stream = torch.cuda.Stream()
    tb = TreeBuilder(S, use_graph)
    best, ms, nn = C.c_int32(0), C.c_float(0.0), C.c_int32(0)
    with torch.cuda.stream(stream) if stream is not None else _nullctx():
        rc = lib().msa_autotune_tree(C.byref(tb.ss), C.byref(tb.ts), C.byref(nn),
                                     int(tb.use_graph), _ptr(tb.ws), tb.wsb, int(reps),
                                     C.byref(best), C.byref(ms), _ptr(tb.st.t), _stream(stream))
    _check(rc, "msa_autotune_tree")
    torch.cuda.synchronize()
    tb.st.check("msa_autotune_tree")
    return best.value, ms.value


def autotune_tree_xl(S: Seqs, pivots: int = 0, topk: int = 16, reps: int = 1, use_graph=True,
                     stream=None):
    """Time the tree build (sampled with `pivots` > 0, else exact) per
    across-lanes variant and keep the fastest in the table; returns (the
    MSA_TUNE_TREE_XL value, ms per build)."""
    if use_graph and stream is None:
        stream = torch.cuda.Stream()
    tb = TreeBuilder(S, use_graph)
    best, ms, nn = C.c_int32(0), C.c_float(0.0), C.c_int32(0)
    with torch.cuda.stream(stream) if stream is not None else _nullctx():
        rc = lib().msa_autotune_tree_xl(C.byref(tb.ss), int(pivots), int(topk), C.byref(tb.ts),
                                        C.byref(nn), int(tb.use_graph), _ptr(tb.ws), tb.wsb,
                                        int(reps), C.byref(best), C.byref(ms), _ptr(tb.st.t),
                                        _stream(stream))
    _check(rc, "msa_autotune_tree_xl")
    torch.cuda.synchronize()
    tb.st.check("msa_autotune_tree_xl")
    return best.value, ms.value


def xl_describe(v: int) -> str:
    """A MSA_TUNE_TREE_XL value as text."""
    wl, pc, sc = v >> 28, (v >> 14) & XL_CAP_ALL, v & XL_CAP_ALL
    cap = lambda c: "all" if c == XL_CAP_ALL else str(c)
    return f"{wl} word(s) per lane, sums up to {cap(sc)}, poles up to {cap(pc)}"


# ---------------------------------------------------------------- embedder
CNN_LAYERS, CNN_WIDTH, CNN_K, CNN_IN = 4, 128, 5, 8


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Embedder:
    """Device parameters of the CNN surrogate (see include/msadp.h)."""

    def __init__(self, dev=None):
        dev = dev or _device()
        self.dev = dev
        self.params = torch.zeros(lib().cnn_param_bytes(), dtype=torch.uint8, device=dev)
        self.step = 0

    def set_params(self, params):
        """params: list of (W[K][cin][128], b[128]) float arrays; layer 0 may
        have cin = sigma (< 8): the extra one-hot channels get zero weights."""
        ws, bs = [], []
        for l, (W, b) in enumerate(params):
            W = np.asarray(W, dtype=np.float32)
            if l == 0 and W.shape[1] < CNN_IN:
                W = np.concatenate([W, np.zeros((W.shape[0], CNN_IN - W.shape[1], W.shape[2]),
                                                np.float32)], axis=1)
            ws.append(W.ravel())
            bs.append(np.asarray(b, dtype=np.float32).ravel())
        w = np.ascontiguousarray(np.concatenate(ws))
        b = np.ascontiguousarray(np.concatenate(bs))
        _check(lib().cnn_set_params(_ptr(self.params), _np_ptr(w), _np_ptr(b),
                                    _stream(None)), "cnn_set_params")
        torch.cuda.synchronize()
        self.step = 0

    def get(self):
        """(params, grads) as lists of (W[K][cin][128], b[128]) float32."""
        sizes = [CNN_K * (CNN_IN if l == 0 else CNN_WIDTH) * CNN_WIDTH for l in range(CNN_LAYERS)]
        w = np.zeros(sum(sizes), np.float32)
        gw = np.zeros(sum(sizes), np.float32)
        b = np.zeros(CNN_LAYERS * CNN_WIDTH, np.float32)
        gb = np.zeros(CNN_LAYERS * CNN_WIDTH, np.float32)
        torch.cuda.synchronize()
        _check(lib().cnn_get_params(_ptr(self.params), _np_ptr(w), _np_ptr(b), _np_ptr(gw),
                                    _np_ptr(gb), _stream(None)), "cnn_get_params")
        out_p, out_g, o = [], [], 0
        for l, n in enumerate(sizes):
            cin = CNN_IN if l == 0 else CNN_WIDTH
            shape = (CNN_K, cin, CNN_WIDTH)
            out_p.append((w[o:o + n].reshape(shape), b[l * CNN_WIDTH:(l + 1) * CNN_WIDTH]))
            out_g.append((gw[o:o + n].reshape(shape), gb[l * CNN_WIDTH:(l + 1) * CNN_WIDTH]))
            o += n
        return out_p, out_g

    def embed(self, S: Seqs, idx=None, chunk=16384, stream=None):
        """float32 embeddings [len(idx), 128] (device tensor)."""
        idx = np.arange(S.n, dtype=np.int32) if idx is None else np.asarray(idx, np.int32)
        out = torch.empty((len(idx), CNN_WIDTH), dtype=torch.float32, device=self.dev)
        ss = S.struct()
        st = Status(self.dev)
        for a in range(0, len(idx), chunk):
            sub = idx[a:a + chunk]
            tl = int(S.lengths[sub].sum())
            wsb = lib().cnn_workspace_bytes(C.byref(ss), len(sub), tl, 0)
            ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=self.dev)
            d_idx = torch.from_numpy(sub).to(self.dev)
            rc = lib().cnn_embed(_ptr(self.params), C.byref(ss), _ptr(d_idx), len(sub), tl,
                                 _ptr(out[a:a + len(sub)]), _ptr(ws), wsb, _ptr(st.t),
                                 _stream(stream))
            _check(rc, "cnn_embed")
        st.check("cnn_embed")
        return out

    def train_step(self, S: Seqs, idx, pa, pb, dist, lr=1e-3, stream=None):
        """One Adam step; returns the batch loss before the update."""
        idx = np.asarray(idx, np.int32)
        tl = int(S.lengths[idx].sum())
        ss = S.struct()
        wsb = lib().cnn_workspace_bytes(C.byref(ss), len(idx), tl, len(pa))
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=self.dev)
        d_idx = torch.from_numpy(idx).to(self.dev)
        d_pa = _i32(pa, self.dev)
        d_pb = _i32(pb, self.dev)
        d_dist = dist if isinstance(dist, torch.Tensor) else \
            torch.from_numpy(np.asarray(dist, np.uint16)).to(self.dev)
        loss = torch.zeros(1, dtype=torch.float32, device=self.dev)
        st = Status(self.dev)
        self.step += 1
        rc = lib().cnn_train_step(_ptr(self.params), C.byref(ss), _ptr(d_idx), len(idx), tl,
                                  _ptr(d_pa), _ptr(d_pb), _ptr(d_dist), len(pa), float(lr),
                                  self.step, _ptr(loss), _ptr(ws), wsb, _ptr(st.t),
                                  _stream(stream))
        _check(rc, "cnn_train_step")
        st.check("cnn_train_step")
        return float(loss.item())


# ---------------------------------------------------------- machine probes
PROBE_MFMA = {"bf16_16x16x32": 0, "bf16_32x32x16": 1, "i8_16x16x64": 2, "i8_32x32x32": 3}


def probe_valu(blocks: int, iters: int, sink: torch.Tensor, stream=None) -> int:
    """Launch the VALU rate probe; returns the lane-instructions it runs."""
    ops = C.c_int64(0)
    _check(lib().msa_probe_valu(int(blocks), int(iters), _ptr(sink), C.byref(ops),
                                _stream(stream)), "msa_probe_valu")
    return ops.value


def probe_mfma(kind: str, blocks: int, iters: int, sink: torch.Tensor, stream=None) -> int:
    """Launch the MFMA rate probe of one shape; returns its operations."""
    ops = C.c_int64(0)
    _check(lib().msa_probe_mfma(PROBE_MFMA[kind], int(blocks), int(iters), _ptr(sink),
                                C.byref(ops), _stream(stream)), "msa_probe_mfma")
    return ops.value


def probe_copy(src: torch.Tensor, dst: torch.Tensor, blocks: int, stream=None) -> int:
    """Launch the streaming copy probe over all of src; returns bytes moved."""
    nb = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() >= nb
    _check(lib().msa_probe_copy(_ptr(src), _ptr(dst), nb, int(blocks), _stream(stream)),
           "msa_probe_copy")
    return 2 * nb
