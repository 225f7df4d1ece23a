"""The hand-written stable radix sort behind the plan's binning of the visibility records and
the bounded solver's breakpoint order (GPU), against numpy's stable argsort: keys bit-exact,
carried values bit-exact (so the order of equal keys is checked too).  Sizes straddle the
launch-shape switches: one partial tile, one full tile, 256 blocks of one round, the first
size with two rounds, the first with eight, and a large ragged size."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2609_17636_amd import sort_u64  # noqa: E402

SIZES = [1, 255, 256, 257, 2047, 65536, 65537, 524288, 524289, 3_000_001]


def _keys(kind, n, rng):
    if kind == "random":
        return rng.integers(0, 2 ** 63, size=n, dtype=np.int64).view(np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, size=n, dtype=np.int64).view(np.uint64)
    if kind == "few":  # many equal keys: stability decides the values' order
        return rng.integers(0, 7, size=n, dtype=np.int64).view(np.uint64) << np.uint64(40)
    if kind == "breakpoints":  # non-negative doubles and +inf, as the solver sorts them
        t = rng.exponential(1.0, size=n) * 10.0 ** rng.integers(-6, 4, size=n)
        t[rng.random(n) < 0.4] = np.inf
        t[rng.random(n) < 0.05] = 0.0
        return t.view(np.uint64)
    raise ValueError(kind)


def _check(keys, end_bit, with_values=True):
    n = keys.size
    mask = np.uint64(0xFFFFFFFFFFFFFFFF) if end_bit == 64 else np.uint64((1 << end_bit) - 1)
    order = np.argsort(keys & mask, kind="stable")
    kt = torch.from_numpy(keys.view(np.int64).copy()).cuda()
    vt = torch.arange(n, dtype=torch.int32, device="cuda") if with_values else None
    ko, vo = sort_u64(kt, vt, end_bit=end_bit)
    torch.cuda.synchronize()
    got_k = ko.cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got_k, keys[order])
    if with_values:
        np.testing.assert_array_equal(vo.cpu().numpy(), order.astype(np.int32))


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kind", ["random", "few", "breakpoints"])
def test_sort_pairs_is_stable_and_exact(n, kind):
    print(f"[sort] n={n} kind={kind}", flush=True)
    _check(_keys(kind, n, np.random.default_rng(n + len(kind))), 64)


@pytest.mark.parametrize("end_bit", [1, 8, 13, 40, 63])
def test_partial_bit_range(end_bit):
    """Only bits [0, end_bit) order the keys; the higher bits travel with them."""
    rng = np.random.default_rng(end_bit)
    _check(_keys("random", 70_001, rng), end_bit)


def test_keys_only_and_empty():
    rng = np.random.default_rng(9)
    _check(_keys("random", 100_003, rng), 64, with_values=False)
    k, v = sort_u64(torch.empty(0, dtype=torch.int64, device="cuda"))
    assert k.numel() == 0 and v is None
