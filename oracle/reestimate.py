"""Final FP64 re-estimation of the recovered coefficients (test infrastructure).

EstimateValues (Algorithm 2) estimates x_i from one hashing as the bin value
divided by the window weight and the shift's phase; applied to x minus the
other recovered coefficients (x - zhat_{-i}) it reads

    e_m(i) = (u_m[h] - sum_{i' != i, h_m(i') = h} c_m(i') v(i')) / c_m(i),

with h = h_m(i) the bin of i in measurement m, c_m(i) = G'_{-o_m(i)} times
omega^{a_m sigma_m i} (the term a coefficient adds to its bin, HashToBins
lemma of Section 3) and v(i') the value taken for the other entry.  A
measurement is valid for i when G'_{-o_m(i)} >= g_min.  The value of i is the
coordinate-wise median of its estimates.

Which value v(i') to subtract is the choice this module makes.  A value
decoded while a not-yet-found neighbour shared its bin carries that
neighbour's window leakage (G' as small as 1e-5 times its magnitude), and
subtracting it passes the error on.  So entries are resolved in passes,
each pass reading only values fixed by earlier passes:

  * pass p (p = 1, 2, ...): an unresolved entry with at least one valid
    measurement in which every other zhat entry of its bin is resolved (in
    pass 1: in which it is alone in its bin, the no-collision case of the
    estimation lemmas) takes the median of its estimates over exactly those
    measurements, subtracting the resolved values; it is resolved from then
    on.  Passes stop when one resolves nothing, or after MAX_PASSES;
  * an entry still unresolved takes the median over all of its valid
    measurements, subtracting resolved values where a neighbour has one and
    the decoded value otherwise;
  * an entry with no valid measurement keeps its decoded value.

On an exactly sparse spectrum whose support is found, every estimate used
in passes is then exact up to the window error delta, whatever order the
coefficients were found in.
"""
from .params import complex_median

MAX_PASSES = 8


def peel_reestimate(zhat, meas, g_min, max_passes=MAX_PASSES):
    """Re-estimated values {i: v} of the zhat entries.

    zhat  {index: decoded value}
    meas  list of measurements (u, terms): u the raw bins of one hashing
          (before any subtraction) and terms {i: (h, g, c)} for every zhat
          entry, with h its bin, g = G'_{-o(i)} and c the complex term
          coefficient (g for exact-mode shift 0, g omega^{a sigma i} in
          general)
    """
    keys = sorted(zhat)
    members = []
    for u, terms in meas:
        by_bin = {}
        for i in keys:
            by_bin.setdefault(terms[i][0], []).append(i)   # ascending index within a bin
        members.append(by_bin)
    valid = {i: [m for m, (u, terms) in enumerate(meas) if terms[i][1] >= g_min] for i in keys}
    resolved = {}

    def estimate(i, m):
        u, terms = meas[m]
        h, g, c = terms[i]
        others = 0.0 + 0.0j
        for i2 in members[m][h]:
            if i2 != i:
                others += terms[i2][2] * resolved.get(i2, zhat[i2])
        return (u[h] - others) / c

    for _ in range(max_passes):
        newly = {}
        for i in keys:
            if i in resolved:
                continue
            ready = [m for m in valid[i]
                     if all(i2 == i or i2 in resolved for i2 in members[m][meas[m][1][i][0]])]
            if ready:
                newly[i] = complex_median([estimate(i, m) for m in ready])
        if not newly:
            break
        resolved.update(newly)
    out = {}
    for i in keys:
        if i in resolved:
            out[i] = resolved[i]
        elif valid[i]:
            out[i] = complex_median([estimate(i, m) for m in valid[i]])
        else:
            out[i] = zhat[i]
    return out
