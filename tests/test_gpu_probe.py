"""pic_probe_stream (the push's particle stream without its arithmetic, a
measurement aid): it reads and writes back six arrays, leaving every value
bit-identical, for sizes that are and are not multiples of its 16,384-value
workgroup slice, with and without the non-temporal hint; it refuses null
arrays."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 16384, 16384 * 3 + 77, 1 << 20])
def test_probe_leaves_the_data_unchanged(n):
    import torch
    from paper_2501_14795_amd import _lib
    g = torch.Generator(device="cuda").manual_seed(n)
    arrays = [torch.randn(n, generator=g, device="cuda") for _ in range(6)]
    before = [a.cpu().numpy().copy() for a in arrays]
    s = torch.cuda.current_stream().cuda_stream
    for nt in (True, False):
        _lib.pic_probe_stream([a.data_ptr() for a in arrays], n, nt, s)
    torch.cuda.synchronize()
    for a, b in zip(arrays, before):
        assert np.array_equal(a.cpu().numpy(), b)
    with pytest.raises(_lib.PicError):
        _lib.pic_probe_stream([arrays[0].data_ptr()] * 5 + [0], n, True, s)


@pytest.mark.parametrize("n", [16384 * 2 + 5, 1 << 20])
def test_probe_with_a_16_bit_first_array(n):
    """The probe's own layout -- arrays[0] of 16-bit values (the cells as
    the push streams them), arrays[1..5] of 32-bit ones, each array exactly
    n values followed by guard values -- with a slice count that is not a
    whole number of workgroup slices: every value, the n streamed and the
    guards, is what it was (a measurement aid must not disturb the data it
    streams)."""
    import torch
    from paper_2501_14795_amd import _lib
    g = torch.Generator(device="cuda").manual_seed(7)
    guard = 4096
    cell = torch.randint(-30000, 30000, (n + guard,), generator=g, device="cuda", dtype=torch.int16)
    rest = [torch.randn(n + guard, generator=g, device="cuda") for _ in range(5)]
    before = [cell.cpu().numpy().copy()] + [a.cpu().numpy().copy() for a in rest]
    s = torch.cuda.current_stream().cuda_stream
    for nt in (True, False):
        _lib.pic_probe_stream([cell.data_ptr()] + [a.data_ptr() for a in rest], n, nt, s)
    torch.cuda.synchronize()
    after = [cell.cpu().numpy()] + [a.cpu().numpy() for a in rest]
    for b, a in zip(before, after):
        assert np.array_equal(a, b)
