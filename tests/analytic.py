"""Closed forms the tests compare with (written from their papers), and the
loader of the values the paper prints (tests/golden/)."""
import os

import numpy as np
from scipy import integrate


def hummer_r2a(x, xp, a):
    """Hummer's (1962) R_II-A redistribution (isotropic angular
    redistribution, coherent in the atom frame), signed form:
    R(x,x') = pi^-3/2 int_{|xbar-xlow|/2}^inf exp(-u^2) [atan((xlow+u)/a) - atan((xbar-u)/a)] du,
    xlow = min(x,x'), xbar = max(x,x').  Normalised over x' it integrates to
    phi(x) = H(a,x)/sqrt(pi)."""
    lo, hi = min(x, xp), max(x, xp)
    f = lambda u: np.exp(-u * u) * (np.arctan((lo + u) / a) - np.arctan((hi - u) / a))
    u0 = abs(hi - lo) / 2.0
    pts = [abs(hi + lo) / 2.0] if abs(hi + lo) / 2.0 < u0 + 8 else None
    v, _ = integrate.quad(f, u0, u0 + 8.0, limit=400, points=pts)
    return v / np.pi ** 1.5


def r2a_expected_counts(x_in, a, edges, n):
    from scipy.special import wofz
    phi = wofz(x_in + 1j * a).real / np.sqrt(np.pi)
    out = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        xm = np.linspace(lo, hi, 5)
        vals = np.array([hummer_r2a(x_in, xp, a) for xp in xm])
        out.append(integrate.simpson(vals, x=xm) / phi * n)
    return np.array(out)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    """Rows of the fixture tests/golden/<name>.txt (values the paper prints,
    cited in the file's header): a list of whitespace-separated fields,
    numbers converted to float."""
    rows = []
    with open(f"{GOLDEN}/{name}.txt") as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            row = []
            for tok in line.split():
                try:
                    row.append(float(tok))
                except ValueError:
                    row.append(tok)
            rows.append(row)
    return rows

