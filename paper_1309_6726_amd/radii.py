"""Effective radius of a reactive capillary from Eq. (1) (section "Results and
discussion", Fig. 4).

At long times the linear Washburn law of Eq. (1) moves the front at
v = gamma H cos(theta) / (6 mu L).  The front velocity of a run is the
least-squares slope of its sampled z(t); a run without reaction fixes
cos(theta) for the capillary, and a reactive run's velocity then gives the
effective width r_eff = 6 mu L v / (gamma cos(theta)), which includes the
retardation by surface growth over the whole run.  (r_min, r_ave and the
hydraulic radius r_h = A / P are observed on the device, `lbm_observe`.)
"""

from __future__ import annotations

import numpy as np


def velocity(t, z, t_min: float = 0.0, t_max: float = np.inf) -> float:
    """Least-squares slope of z(t) over the samples with t_min <= t <= t_max."""
    t = np.asarray(t, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    sel = (t >= t_min) & (t <= t_max) & np.isfinite(z)
    if np.count_nonzero(sel) < 2:
        raise ValueError("need at least two samples")
    tt, zz = t[sel], z[sel]
    tc = tt - tt.mean()
    return float(np.dot(tc, zz - zz.mean()) / np.dot(tc, tc))


def cos_theta(v0: float, H: float, L: float, gamma: float, mu: float) -> float:
    """cos(theta) that makes Eq. (1) reproduce the no-reaction velocity v0."""
    return 6.0 * mu * L * v0 / (gamma * H)


def r_eff(t, z, L: float, gamma: float, mu: float, cos_t: float, **window) -> float:
    """Width for which Eq. (1) gives the run's least-squares front velocity."""
    return 6.0 * mu * L * velocity(t, z, **window) / (gamma * cos_t)
