"""GPU checks of the dense-path selection (sfft_dense_topk) against a numpy
selection on the same keys.  Spectra have small-integer components, so every
key |X|^2 is exact and ties are everywhere: the cap largest keys, ties to
the smaller index, ascending indices, values times scale, unused slots zero;
the keep_above filter; the whole spectrum (cap >= n); an all-zero spectrum;
batches whose tied bins span many of the selection's chunks.  Every case
prints its name before touching the GPU."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1201_2501_amd import sfft
    sfft.load()
    return torch, torch.device("cuda:0"), sfft


def ref_topk(X, cap, scale, keep_above):
    key = X.real.astype(np.float64) ** 2 + X.imag.astype(np.float64) ** 2     # exact for small integers
    order = np.lexsort((np.arange(len(X)), -key))[:cap]
    if keep_above >= 0:
        kt = float(np.float32((keep_above / scale) * (keep_above / scale)))
        order = order[key[order] > kt]
    order = np.sort(order)
    return order, X[order].astype(np.complex128) * scale


def int_spectrum(rng, n, lo, hi, plant_every=0, plant=3 + 3j):
    X = (rng.integers(lo, hi + 1, n) + 1j * rng.integers(lo, hi + 1, n)).astype(np.complex64)
    if plant_every:
        X[::plant_every] = plant
    return X


def check(env, name, spectra, cap, scale, keep_above=-1.0):
    torch, dev, sfft = env
    S = np.stack(spectra).astype(np.complex64)
    say("dense-topk", name, "count", S.shape[0], "n", S.shape[1], "cap", cap, "keep_above", keep_above)
    idx, val, cnt = sfft.dense_topk(torch.from_numpy(S).to(dev), cap, scale, keep_above)
    torch.cuda.synchronize()
    idx, val, cnt = idx.cpu().numpy(), val.cpu().numpy(), cnt.cpu().numpy()
    for s in range(S.shape[0]):
        ri, rv = ref_topk(S[s], cap, scale, keep_above)
        c = int(cnt[s])
        assert c == len(ri), (name, s, c, len(ri))
        assert np.array_equal(idx[s, :c], ri), name
        assert np.array_equal(val[s, :c], rv), name
        assert not idx[s, c:].any() and not val[s, c:].any()


def test_ties_within_one_chunk(env):
    rng = np.random.default_rng(1)
    check(env, "one-chunk", [int_spectrum(rng, 1 << 12, -3, 3) for _ in range(3)], 100, 1.0 / 64)


def test_ties_across_chunks(env):
    # 1,772 planted maxima every 37th bin of 2^16: the 1000 taken span 9 chunks
    rng = np.random.default_rng(2)
    check(env, "16-chunks", [int_spectrum(rng, 1 << 16, -1, 1, plant_every=37) for _ in range(2)], 1000, 0.25)


def test_ties_across_many_chunks_large_n(env):
    # 2^20 bins (256 chunks), 1,052 planted maxima every 997th bin: 1024 taken
    rng = np.random.default_rng(3)
    check(env, "256-chunks", [int_spectrum(rng, 1 << 20, -2, 2, plant_every=997, plant=4 - 4j),
                              int_spectrum(rng, 1 << 20, -2, 2)], 1024, 1.0 / 1024)


def test_largest_chunk_layout(env):
    # 2^24 bins: 1024 chunks of 16,384; 1,023 planted maxima every 16,411th bin, the first 1,000 taken
    rng = np.random.default_rng(6)
    check(env, "2^24", [int_spectrum(rng, 1 << 24, -1, 1, plant_every=16411, plant=2 + 2j)], 1000, 2.0 ** -12)


def test_keep_above_filters_on_the_key(env):
    # keys of components in [-2, 2] are 0, 1, 2, 4, 5, 8; the threshold's key is 4.5
    rng = np.random.default_rng(4)
    scale = 0.5
    # 2^13 bins: about 3,900 keys above 4.5, so the 6,000 selected reach keys 4 and 2 that the filter drops
    check(env, "keep-above", [int_spectrum(rng, 1 << 13, -2, 2) for _ in range(2)], 6000, scale,
          keep_above=np.sqrt(4.5) * scale)


def test_whole_spectrum_and_zero_spectrum(env):
    rng = np.random.default_rng(5)
    X = int_spectrum(rng, 1 << 10, -1, 1)
    check(env, "cap=n", [X], 1 << 10, 1.0)
    check(env, "cap=n keep", [X], 1 << 10, 1.0, keep_above=0.5)
    Z = np.zeros(1 << 12, np.complex64)
    check(env, "zeros", [Z], 50, 1.0)
    check(env, "zeros keep", [Z], 50, 1.0, keep_above=0.0)


def test_rejects_bad_arguments(env):
    torch, dev, sfft = env
    x = torch.zeros((1, 1000), dtype=torch.complex64, device=dev)
    with pytest.raises(RuntimeError):
        sfft.dense_topk(x, 10, 1.0)                 # n not a power of two
    y = torch.zeros((1, 1 << 10), dtype=torch.complex64, device=dev)
    with pytest.raises(RuntimeError):
        sfft.dense_topk(y, 0, 1.0)                  # cap 0
