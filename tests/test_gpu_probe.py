"""The streaming reference kernels (hmc_stream_probe) move what they claim: the read forms sum
every element once (plain and nontemporal loads), the write form writes each vector's index,
copy and 3r3w write 1.5 times each source stream; a ragged grid (more workgroups than vectors
per pass) and a size that is not a multiple of the grid's span are covered."""
import sys

import pytest
import torch

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("grid", [1, 7, 2048])
def test_read_forms_sum_every_element_once(hip, grid):
    n4 = 3 * 256 * 8 + 5                    # 16-byte vectors; not a multiple of any span
    src = torch.ones(4 * n4, dtype=torch.float32, device="cuda")
    for kind in ("read", "read_nt"):
        part = torch.zeros(grid, dtype=torch.float64, device="cuda")
        hip.stream_probe(kind, src, part, 16 * n4, grid)
        torch.cuda.synchronize()
        say(f"probe {kind} grid {grid}: sum {part.sum().item()} of {4 * n4}")
        assert part.sum().item() == 4 * n4


@pytest.mark.parametrize("grid", [3, 2048])
def test_write_copy_and_3r3w_forms(hip, grid):
    n4 = 256 * 5 + 3
    dst = torch.zeros(4 * n4, dtype=torch.float32, device="cuda")
    hip.stream_probe("write", None, dst, 16 * n4, grid)
    idx = torch.arange(n4, dtype=torch.float32, device="cuda").repeat_interleave(4)
    assert torch.equal(dst, idx)
    src = torch.randn(3 * 4 * n4, dtype=torch.float32, device="cuda")
    out = torch.zeros(3 * 4 * n4, dtype=torch.float32, device="cuda")
    hip.stream_probe("copy", src, out, 16 * n4, grid)
    assert torch.equal(out[:4 * n4], 1.5 * src[:4 * n4]) and not out[4 * n4:].any()
    hip.stream_probe("3r3w", src, out, 16 * n4, grid)
    torch.cuda.synchronize()
    assert torch.equal(out, 1.5 * src)
