"""Small numpy helpers shared by the tests (error norms of Sec. 5, golden-file reader)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    return np.array(rows)


def norm_n(F):
    """||F||_N = sqrt(<F, F>_N) for a field [3, nz, ny, nx] (grid mean, components summed)."""
    return float(np.sqrt(np.mean(np.sum(np.asarray(F) ** 2, axis=0))))


def errors(H, E, Hx, Ex):
    """(L_inf, L_2) of Sec. 5: max abs error, and sqrt(||dE||_N^2 + ||dH||_N^2)."""
    dH = np.asarray(H) - Hx
    dE = np.asarray(E) - Ex
    linf = max(float(np.max(np.abs(dH))), float(np.max(np.abs(dE))))
    l2 = float(np.sqrt(norm_n(dH) ** 2 + norm_n(dE) ** 2))
    return linf, l2


def energy_rel_error(H, E, Hx, Ex, mu, eps):
    """Error in the energy norm of Thm 3.4, relative to the norm of the exact state."""
    num = mu * norm_n(np.asarray(H) - Hx) ** 2 + eps * norm_n(np.asarray(E) - Ex) ** 2
    den = mu * norm_n(Hx) ** 2 + eps * norm_n(Ex) ** 2
    return float(np.sqrt(num / den))


def elementwise_rel_error(H, E, Hx, Ex, mu, eps):
    """Largest pointwise error over all six components, relative to the largest value
    of the reference, both in the energy weighting (sqrt(mu) H, sqrt(eps) E).  A local
    mistake (one bad tile, plane or pencil) shows here even when it barely moves the
    global energy norm."""
    sm, se = float(np.sqrt(mu)), float(np.sqrt(eps))
    err = max(sm * float(np.max(np.abs(np.asarray(H) - Hx))), se * float(np.max(np.abs(np.asarray(E) - Ex))))
    ref = max(sm * float(np.max(np.abs(Hx))), se * float(np.max(np.abs(Ex))))
    return err / ref
