"""Machine-rate probes: the copy probe copies exactly, and the work counts
the probes report match their stated instruction counts."""
import pytest
import torch

from paper_2601_15458_amd import msadp

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes,blocks", [(16, 1), (4096 * 16 + 48, 7), (1 << 22, 64),
                                           ((1 << 24) + 16 * 1001, 4096)])
def test_copy_probe_copies(nbytes, blocks):
    g = torch.Generator().manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    moved = msadp.probe_copy(src, dst[:nbytes], blocks)
    torch.cuda.synchronize()
    assert moved == 2 * nbytes
    assert torch.equal(dst[:nbytes], src)
    assert int(dst[nbytes:].count_nonzero()) == 0


def test_valu_probe_work_count():
    sink = torch.zeros(3 * 256, dtype=torch.int32, device="cuda")
    ops = msadp.probe_valu(3, 5, sink)
    torch.cuda.synchronize()
    assert ops == 128 * 5 * 3 * 256
    assert int(sink.count_nonzero()) > 0          # every lane wrote its chain result


@pytest.mark.parametrize("kind,mnk", [("bf16_16x16x32", 16 * 16 * 32),
                                      ("bf16_32x32x16", 32 * 32 * 16),
                                      ("i8_16x16x64", 16 * 16 * 64),
                                      ("i8_32x32x32", 32 * 32 * 32)])
def test_mfma_probe_work_count(kind, mnk):
    sink = torch.zeros(2 * 256, dtype=torch.int32, device="cuda")
    ops = msadp.probe_mfma(kind, 2, 3, sink)
    torch.cuda.synchronize()
    # 2 blocks x 4 wavefronts x 3 trips x 16 instructions x 2 M N K
    assert ops == 2 * 4 * 3 * 16 * 2 * mnk
