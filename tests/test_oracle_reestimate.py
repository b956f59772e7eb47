"""Pins of the final re-estimation (EstimateValues of Algorithm 2 applied to
x minus the other recovered coefficients, resolved in passes).

The measurements here are built by hand from a known spectrum, so the exact
values are known: u_m[h] = sum over the bin of c_m(i) x_i."""
import numpy as np
import pytest

from oracle.reestimate import peel_reestimate


def bins_of(x, layout):
    """Raw bins of one measurement: layout {i: (h, g, c)}."""
    nb = 1 + max(h for h, _, _ in layout.values())
    u = np.zeros(nb, complex)
    for i, (h, g, c) in layout.items():
        u[h] += c * x[i]
    return u


def test_leaked_neighbour_is_resolved_first():
    """Entry 1 is never alone where it is valid; entry 0 is alone once.  Its
    decoded value is off by leakage; the result must still be exact."""
    x = {0: 2.0 - 1.0j, 1: 0.5 + 0.25j, 2: -1.0 + 0.0j}
    meas = [
        {0: (0, 1.0, 1.0), 1: (0, 1e-5, 1e-5), 2: (1, 1.0, 1.0)},   # 1 leaks into 0's bin
        {0: (1, 0.9, 0.9), 1: (1, 1.0, 1.0), 2: (0, 0.8, 0.8)},     # 0 and 1 share
        {0: (0, 1.0, 1.0), 1: (0, 0.7, 0.7), 2: (2, 1.0, 1.0)},     # 0 and 1 share
        {0: (3, 1.0, 1.0), 1: (2, 0.1, 0.1), 2: (1, 0.6, 0.6)},     # 0 alone, 1 invalid
    ]
    m = [(bins_of(x, lay), lay) for lay in meas]
    zhat = {0: x[0] + 1e-5 * x[1], 1: x[1] + 3e-4, 2: x[2] + 1e-3}
    out = peel_reestimate(zhat, m, g_min=0.4)
    for i in x:
        assert abs(out[i] - x[i]) < 1e-14, (i, out[i], x[i])


def test_single_pass_would_keep_the_leak():
    """The same data with the neighbour's decoded value subtracted (one pass,
    no resolution order) is off by the leak: the pin above is not vacuous."""
    x = {0: 2.0 - 1.0j, 1: 0.5 + 0.25j}
    lay = [{0: (0, 1.0, 1.0), 1: (0, 0.7, 0.7)}, {0: (1, 1.0, 1.0), 1: (0, 0.1, 0.1)}]
    m = [(bins_of(x, l), l) for l in lay]
    zhat = {0: x[0] + 1e-3, 1: x[1]}
    direct = (m[0][0][0] - 1.0 * zhat[0]) / 0.7     # entry 1 from the shared bin, decoded neighbour
    assert abs(direct - x[1]) > 1e-4
    out = peel_reestimate(zhat, m, g_min=0.4)
    assert abs(out[1] - x[1]) < 1e-14 and abs(out[0] - x[0]) < 1e-14


def test_complex_term_coefficients_and_median():
    """General-mode terms c = G' omega^{a sigma i}: estimates divide by c; the
    median over an odd count of alone measurements ignores one outlier."""
    rng = np.random.default_rng(3)
    x = {5: 1.0 + 2.0j}
    lays = []
    for _ in range(5):
        ph = np.exp(2j * np.pi * rng.random())
        g = 0.5 + 0.5 * rng.random()
        lays.append({5: (0, g, g * ph)})
    m = [(bins_of(x, l), l) for l in lays]
    m[2] = (m[2][0] + 10.0, m[2][1])                   # one corrupted bin
    out = peel_reestimate({5: 0.0 + 0.0j}, m, g_min=0.4)
    assert abs(out[5] - x[5]) < 1e-14


def test_unresolvable_pair_falls_back_to_all_valid_measurements():
    """Two entries sharing every valid bin cannot be peeled: each takes the
    median over all its valid measurements with the other's decoded value."""
    x = {0: 1.0 + 0.0j, 1: 0.0 + 1.0j}
    lays = [{0: (0, 1.0, 1.0), 1: (0, 0.5, 0.5)}, {0: (0, 0.6, 0.6), 1: (0, 1.0, 1.0)},
            {0: (0, 0.9, 0.9), 1: (0, 0.9, 0.9)}]
    m = [(bins_of(x, l), l) for l in lays]
    zhat = {0: x[0] + 0.01, 1: x[1] - 0.02}
    out = peel_reestimate(zhat, m, g_min=0.4)
    e0 = sorted(((m[q][0][0] - lays[q][1][2] * zhat[1]) / lays[q][0][2]).real for q in range(3))
    assert abs(out[0].real - e0[1]) < 1e-14
    assert abs(out[0] - x[0]) > 1e-3                   # not exact: no order resolves them


def test_no_valid_measurement_keeps_the_decoded_value():
    lay = [{7: (0, 0.1, 0.1)}]
    out = peel_reestimate({7: 3.0 + 1.0j}, [(np.array([5.0 + 0j]), lay[0])], g_min=0.4)
    assert out[7] == 3.0 + 1.0j


@pytest.mark.parametrize("passes", [1, 2])
def test_pass_cap_limits_chain_depth(passes):
    """A chain 0 -> 1 -> 2, each entry resolvable only after the previous:
    pass 1 resolves 0 and pass 2 resolves 1; the fallback for 2 then
    subtracts 1's resolved value.  With one pass the fallback for 2 has to
    use 1's decoded value and keeps its error."""
    x = {0: 1.0 + 0j, 1: 2.0 + 0j, 2: 3.0 + 0j}
    lays = [{0: (0, 1.0, 1.0), 1: (1, 0.2, 0.2), 2: (2, 0.1, 0.1)},    # 0 alone
            {0: (0, 0.3, 0.3), 1: (0, 1.0, 1.0), 2: (1, 0.1, 0.1)},    # 1 with 0
            {0: (1, 0.1, 0.1), 1: (0, 0.3, 0.3), 2: (0, 1.0, 1.0)}]    # 2 with 1
    m = [(bins_of(x, l), l) for l in lays]
    zhat = {0: 1.1 + 0j, 1: 2.2 + 0j, 2: 3.3 + 0j}
    full = peel_reestimate(zhat, m, g_min=0.4)
    assert all(abs(full[i] - x[i]) < 1e-14 for i in x)
    capped = peel_reestimate(zhat, m, g_min=0.4, max_passes=passes)
    assert abs(capped[0] - x[0]) < 1e-14
    assert abs(capped[1] - x[1]) < 1e-14
    assert (abs(capped[2] - x[2]) > 1e-3) == (passes < 2)
