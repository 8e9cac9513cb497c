"""The seeded input generators (no arithmetic of the method): the
column-major generator of the large workload follows the column-density
law."""
import numpy as np

import synth


def test_column_law_csc_follows_the_law():
    """The column-major generator: rows sorted and distinct in every column,
    column counts Binomial(n, d_j) (standardised counts have mean ~0 and
    spread ~1), rows uniform (a column's rows pass a KS test against
    U[0, n))."""
    from scipy import stats
    n, p = 50_000, 4000
    rng = np.random.default_rng(3)
    dens = np.exp(np.random.default_rng(3).uniform(np.log(1e-4), np.log(0.2), size=p))
    cp, ri = synth.column_law_csc(n, p, rng)
    assert cp[0] == 0 and cp[-1] == ri.size and np.all(np.diff(cp) >= 0)
    for j in range(p):
        r = ri[cp[j]:cp[j + 1]]
        assert np.all(np.diff(r) > 0) and (r.size == 0 or (r[0] >= 0 and r[-1] < n))
    k = np.diff(cp)
    zs = (k - n * dens) / np.sqrt(n * dens * (1 - dens))
    assert abs(zs.mean()) < 0.1 and 0.9 < zs.std() < 1.1
    big = int(np.argmax(k))
    assert stats.kstest(ri[cp[big]:cp[big + 1]] / n, "uniform").pvalue > 1e-3
