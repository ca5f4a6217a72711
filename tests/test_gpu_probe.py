"""GPU: the LDS histogram ceiling probe (a measurement utility) does every
atomic it is asked for: each block's histogram total is the sum of its
added values, steps x learners x 8 x (1 + 2 + ... + 1024)."""
import numpy as np
import pytest

from paper_2110_03513_amd import cwb

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("word_bytes", [4, 8])
@pytest.mark.parametrize("nb,learners,steps,blocks", [(1000, 4, 3, 7), (17, 1, 5, 3), (8192, 2, 1, 2)])
def test_probe_checksums(nb, learners, steps, blocks, word_bytes):
    import torch
    rng = np.random.default_rng(nb)
    tab = rng.integers(0, nb + 50, size=8 * 1024).astype(np.int16)  # some past nb: clamped
    idx = torch.from_numpy(tab).cuda()
    out = torch.zeros(blocks, dtype=torch.int64, device="cuda")
    print(f"probe nb={nb} learners={learners} steps={steps} blocks={blocks} words={word_bytes}",
          flush=True)
    cwb.probe_lds_hist(idx, nb, learners, steps, blocks, out, word_bytes=word_bytes)
    torch.cuda.synchronize()
    want = steps * learners * 8 * (1024 * 1025 // 2)
    assert out.cpu().tolist() == [want] * blocks


def test_probe_rejects_bad_sizes():
    import torch
    idx = torch.zeros(8 * 3, dtype=torch.int16, device="cuda")  # 3 chunks: not a power of two
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(cwb.CwbError):
        cwb.probe_lds_hist(idx, 100, 1, 1, 1, out)
    idx = torch.zeros(8 * 4, dtype=torch.int16, device="cuda")
    with pytest.raises(cwb.CwbError):
        cwb.probe_lds_hist(idx, 8192, 4, 1, 1, out)  # 256 KiB of LDS
