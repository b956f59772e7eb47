"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol that include/sfft.h declares, and its pure host functions agree
with the oracle's independent implementations."""
import os
import re

import pytest

from paper_1201_2501_amd import sfft

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "sfft.h")).read()
    return sorted(set(re.findall(r"\b(sfft_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(sfft.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = sfft.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_splitmix64_matches_golden_vectors():
    from tests.test_oracle_rng import golden_rows
    for seed, c, expect in golden_rows():
        assert sfft.sfft_splitmix64(seed, c) == expect


def test_desc_defaults():
    d = sfft.sfft_desc_init(1 << 22, 256, 1024, 0, 7)
    assert (d.n, d.k, d.B, d.w, d.seed) == (1 << 22, 256, 1024, 0, 7)
    assert d.mode == sfft.SFFT_MODE_EXACT and d.in_dtype == sfft.SFFT_C64
    assert d.loc_prec == sfft.SFFT_F64          # n >= 2^20: FP64 location decoding
    assert sfft.sfft_desc_init(1 << 14, 16, 64).loc_prec == sfft.SFFT_F32
    assert d.alpha == 0.5 and d.patience == 3 and d.rounds == 0     # 0 = mode default
    assert sfft.sfft_validate_params(d) == sfft.SFFT_OK


@pytest.mark.parametrize("field,value,status", [
    ("n", 3000, sfft.SFFT_ENOTPOW2), ("n", 2, sfft.SFFT_ENOTPOW2), ("k", 0, sfft.SFFT_EINVAL),
    ("B", 1000, sfft.SFFT_ENOTPOW2), ("B", 1 << 23, sfft.SFFT_EINVAL), ("w", 1000, sfft.SFFT_EINVAL),
    ("alpha", 1.5, sfft.SFFT_EINVAL), ("delta", 0.0, sfft.SFFT_EINVAL), ("mode", 7, sfft.SFFT_EINVAL),
    ("rounds", 33, sfft.SFFT_EINVAL), ("b_min", 3, sfft.SFFT_EINVAL), ("max_batch", 0, sfft.SFFT_EINVAL),
    ("in_dtype", 5, sfft.SFFT_EINVAL), ("g_min", 0.0, sfft.SFFT_EINVAL),
])
def test_validation_errors(field, value, status):
    d = sfft.sfft_desc_init(1 << 22, 256, 1024, 0, 7)
    setattr(d, field, value)
    assert sfft.sfft_validate_params(d) == status
    assert sfft.sfft_last_error() != ""


def test_general_mode_validation():
    d = sfft.sfft_desc_init(1 << 20, 64, 1024, 0, 7)
    d.mode = sfft.SFFT_MODE_GENERAL
    assert sfft.sfft_validate_params(d) == sfft.SFFT_OK
    d.t = 12
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL
    d.t = 16
    d.rounds, d.R_est = 10, 7
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL        # 70 measurements > 64
    d.rounds = 5
    d.k = 2000
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EUNSUPPORTED  # zhat capacity


def test_lds_limit_is_reported_as_unsupported():
    d = sfft.sfft_desc_init(1 << 22, 256, 8192, 0, 7)
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EUNSUPPORTED
    d.B = 4096
    assert sfft.sfft_validate_params(d) == sfft.SFFT_OK


@pytest.mark.parametrize("n,B,alpha,delta", [(1 << 14, 64, 0.5, 1e-12), (1 << 20, 1024, 0.5, 1e-6),
                                             (1 << 16, 256, 0.25, 1e-9)])
def test_default_window_matches_oracle_definition(n, B, alpha, delta):
    from oracle.window import default_w
    assert sfft.sfft_default_w(n, B, alpha, delta) == default_w(n, B, alpha, delta)


def test_status_strings():
    assert sfft.sfft_status_string(sfft.SFFT_ETRUNC) == "SFFT_ETRUNC"


def test_plan_queries_reject_null_plan():
    import ctypes
    lib = sfft.load()
    ng = ctypes.c_uint32(99)
    assert lib.sfft_plan_round_groups(None, None, 0, ctypes.byref(ng)) == sfft.SFFT_EINVAL
    assert ng.value == 99
    assert lib.sfft_plan_h2b_bytes(None, 4) == 0


def test_general_mode_measurement_limits():
    d = sfft.sfft_desc_init(1 << 20, 64, 1024, 0, 7)
    d.mode = sfft.SFFT_MODE_GENERAL
    d.R_loc = 8
    assert sfft.sfft_validate_params(d) == sfft.SFFT_OK
    d.R_loc = 9
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL
    d.R_loc, d.R_est, d.rounds = 3, 33, 1
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL


def test_general_default_rounds():
    # rounds 0 = max(7, ceil(log4 k) + 2): 7 rounds up to k = 1024, so 10 measurements per round exceed 64
    d = sfft.sfft_desc_init(1 << 22, 1024, 4096, 0, 7)
    d.mode = sfft.SFFT_MODE_GENERAL
    d.R_est = 9
    assert sfft.sfft_validate_params(d) == sfft.SFFT_OK       # 7 * 9 = 63
    d.R_est = 10
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL   # 70
    d.k, d.B = 8, 1024
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL   # still 7 rounds at small k
    d.rounds = 6
    assert sfft.sfft_validate_params(d) == sfft.SFFT_OK       # 6 * 10 given explicitly


def test_hash_split_validation():
    d = sfft.sfft_desc_init(1 << 20, 64, 256)
    d.hash_split = 8
    assert sfft.sfft_validate_params(d) == sfft.SFFT_OK
    d.hash_split = 65
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL
    d.hash_split, d.chunks = 8, 2
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL
    d.chunks, d.mode = 1, sfft.SFFT_MODE_GENERAL
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL
    d.mode, d.hash_mode = sfft.SFFT_MODE_EXACT, 3
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL


def test_plan_desc_layout_matches_the_library():
    assert sfft.load().sfft_plan_desc_bytes() == __import__("ctypes").sizeof(sfft.PlanDesc)


def test_refine_validation():
    d = sfft.sfft_desc_init(1 << 22, 256, 1024)
    d.refine_shift = 2048
    assert sfft.sfft_validate_params(d) == sfft.SFFT_OK              # E = 16 by default
    d.refine_window = 1000
    assert sfft.sfft_validate_params(d) == sfft.SFFT_OK              # 2048 * 2001 < 2^22
    d.refine_window = 1024
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL          # 2048 * 2049 >= 2^22
    d.refine_shift = 16
    assert sfft.sfft_validate_params(d) == sfft.SFFT_OK
    d.refine_window = 1025
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL          # E at most 1024
    d.refine_window, d.refine_shift = 64, (1 << 22) // 129
    assert sfft.sfft_validate_params(d) == sfft.SFFT_OK              # A (2E + 1) = n - 127
    d.refine_shift += 1
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL          # A (2E + 1) >= n
    d.refine_shift = 1
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL
    d.refine_shift = 2048
    for field, value in (("hash_split", 4), ("hash_mode", 1), ("mode", sfft.SFFT_MODE_GENERAL)):
        setattr(d, field, value)
        assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL, field
        setattr(d, field, 0)
    assert sfft.sfft_validate_params(d) == sfft.SFFT_OK


def test_refine_adds_its_samples():
    """The refinement hashing reads A more samples per round for A < w_r + 1
    (one window [t0 - A, t0 + w_r)), else another w_r."""
    d = sfft.sfft_desc_init(1 << 22, 256, 1024, 0, 7)
    d.b_min, d.rounds, d.group0 = 1024, 4, 4                         # four rounds of w
    base = sfft.sfft_plan_samples(d)
    w = sfft.sfft_default_w(1 << 22, 1024, 0.5, d.delta)
    assert base == 4 * (w + 1)
    d.refine_shift = 1000
    assert sfft.sfft_plan_samples(d) == 4 * (w + 1000)
    d.refine_shift, d.refine_window = w + 5, 2
    assert sfft.sfft_plan_samples(d) == 4 * (2 * w + 1)


@pytest.mark.parametrize("n,B,alpha,delta", [(1 << 14, 64, 0.5, 1e-12), (1 << 22, 1024, 0.75, 1e-8),
                                             (1 << 20, 256, 0.6, 1e-7), (1 << 26, 4096, 0.5, 1e-6),
                                             (1 << 12, 1024, 0.5, 1e-9)])
def test_kaiser_window_length_matches_oracle(n, B, alpha, delta):
    from oracle.window import default_w
    assert sfft.sfft_window_w(n, B, alpha, delta, 1) == default_w(n, B, alpha, delta, kind=1)
    assert sfft.sfft_window_w(n, B, alpha, delta, 0) == sfft.sfft_default_w(n, B, alpha, delta)
    assert sfft.sfft_window_w(n, B, alpha, delta, 2) == 0


def test_window_field_validation_and_default_length():
    d = sfft.sfft_desc_init(1 << 22, 256, 1024)
    d.window = 2
    assert sfft.sfft_validate_params(d) == sfft.SFFT_EINVAL
    d.window = 1
    assert sfft.sfft_validate_params(d) == sfft.SFFT_OK
    d.b_min, d.rounds, d.group0 = 1024, 4, 4
    w = sfft.sfft_window_w(1 << 22, 1024, d.alpha, d.delta, 1)
    assert sfft.sfft_plan_samples(d) == 4 * (w + 1)          # w = 0 resolves to the Kaiser length
