"""fftcg_stream_probe (the HBM streaming kernels the benchmark takes its
practical ceiling from): the copy and write kernels move exactly the bytes
asked for, including a ragged tail shorter than one unrolled step, the read
kernel leaves its sink alone on zero data, and bad arguments are rejected."""

import numpy as np
import pytest
import torch

from paper_1305_3625_amd import binding
from gpu_util import banner

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nt", [False, True])
def test_probe_kernels_move_the_bytes(nt):
    n = (1 << 20) + 6          # doubles: 8 MiB + 48 bytes (a ragged tail)
    nbytes = (n - 2) * 8       # a multiple of 16 bytes, leaving 2 sentinels
    banner("stream-probe", nt)
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    ms = binding.stream_probe(2, dst, src, nbytes, 37, reps=2, nontemporal=nt)
    assert ms > 0.0
    got = dst.cpu().numpy()
    assert np.array_equal(got[:n - 2], np.arange(n - 2, dtype=np.float64))
    assert np.all(got[n - 2:] == -1.0)
    binding.stream_probe(1, dst, src, nbytes, 1024, reps=1, nontemporal=nt)
    got = dst.cpu().numpy()
    assert not got[:n - 2].any() and np.all(got[n - 2:] == -1.0)
    zeros = torch.zeros(n, dtype=torch.float64, device="cuda")
    sink = torch.full((2,), 7.0, dtype=torch.float64, device="cuda")
    binding.stream_probe(0, sink, zeros, nbytes, 512, reps=2, nontemporal=nt)
    assert np.all(sink.cpu().numpy() == 7.0)


def test_probe_rejects_bad_arguments():
    a = torch.zeros(64, dtype=torch.float64, device="cuda")
    b = torch.zeros(64, dtype=torch.float64, device="cuda")
    for kind, nbytes, blocks in [(3, 256, 4), (-1, 256, 4), (2, 0, 4), (2, 24, 4), (2, 256, 0)]:
        with pytest.raises(binding.FftcgError):
            binding.stream_probe(kind, a, b, nbytes, blocks, reps=1)
    with pytest.raises(binding.FftcgError):   # overlapping copy
        binding.stream_probe(2, a[2:], a, 256, 4, reps=1)
    with pytest.raises(binding.FftcgError):   # not 16-byte aligned
        binding.stream_probe(2, a[1:], b, 256, 4, reps=1)
