"""The library's stable radix sort (tpe_sort_pairs) against NumPy's stable argsort, bit-exact:
one to many 2,048-key tiles, ragged sizes, every key width (one to four passes), keys with bits
above the sorted ones."""
import numpy as np
import pytest

from tests.gpu_util import log, needs_gpu, tpe

pytestmark = [pytest.mark.gpu, needs_gpu]

SIZES = [2, 63, 64, 65, 1000, 1024, 1025, 20480, 32767, 32768, 32769, 100_000, 300_000]


def run(T, keys_u32, bits):
    import torch
    k = torch.from_numpy(keys_u32.view(np.int32).copy()).cuda()
    v = torch.arange(keys_u32.shape[0], dtype=torch.int32, device="cuda")
    T.sort_pairs(k, v, bits)
    return k.cpu().numpy().view(np.uint32), v.cpu().numpy()


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("bits", [1, 5, 9, 13, 18, 24, 32])
def test_stable_sort(n, bits):
    T = tpe()
    rng = np.random.default_rng(n * 37 + bits)
    mask = np.uint32(0xFFFFFFFF if bits == 32 else (1 << bits) - 1)
    # few distinct low values (many ties), and random bits above the sorted ones
    low = rng.integers(0, min(1 << bits, max(2, n // 3)), n, dtype=np.uint64).astype(np.uint32)
    high = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32) & ~mask
    keys = (low | high).astype(np.uint32)
    ko, vo = run(T, keys, bits)
    order = np.argsort(keys & mask, kind="stable")
    ok = np.array_equal(vo, order) and np.array_equal(ko, keys[order])
    if not ok:
        log("sort mismatch n", n, "bits", bits, "first bad", int(np.argmax(vo != order)))
    assert ok


def test_morton_like_keys_and_errors():
    T = tpe()
    rng = np.random.default_rng(5)
    keys = rng.integers(0, 1 << 18, 20480, dtype=np.uint64).astype(np.uint32)
    ko, vo = run(T, keys, 18)
    assert np.array_equal(vo, np.argsort(keys, kind="stable"))
    import torch
    k = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(T.TPEError):
        T.sort_pairs(k, k.clone(), 0)
    with pytest.raises(ValueError):
        T.sort_pairs(k, torch.zeros(5, dtype=torch.int32, device="cuda"), 8)
