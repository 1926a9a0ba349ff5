"""Post-processing of moment fields: droplets on the plates and per-field
differences between two runs.  Host-side numpy/scipy; not part of the step."""
from __future__ import annotations

import numpy as np
from scipy import ndimage


def _periodic_labels(liq: np.ndarray):
    """4-neighbour labels of a mask, joined across the periodic x boundary."""
    ny, nx = liq.shape
    lab, n = ndimage.label(liq)
    parent = list(range(n + 1))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for y in range(ny):
        a, b = lab[y, 0], lab[y, nx - 1]
        if a and b:
            ra, rb = find(a), find(b)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(i) for i in range(n + 1)])
    return roots[lab]


def liquid_sets(rho: np.ndarray, threshold: float):
    """Connected liquid sets of a plate field rho[y, x] (plate rows included,
    periodic in x), largest first, each as [node count, centroid y, centroid x
    (circular mean), reaches the row below the top plate, reaches the row
    above the bottom plate]."""
    ny, nx = rho.shape
    liq = rho > threshold
    liq[0] = liq[-1] = False
    lab = _periodic_labels(liq)
    out = []
    for i in np.unique(lab[lab > 0]):
        ys, xs = np.nonzero(lab == i)
        ang = 2 * np.pi * xs / nx
        cx = (np.arctan2(np.sin(ang).mean(), np.cos(ang).mean()) % (2 * np.pi)) * nx / (2 * np.pi)
        out.append([int(ys.size), float(ys.mean()), float(cx), int(ys.max() == ny - 2),
                    int(ys.min() == 1)])
    out.sort(key=lambda r: -r[0])
    return out


def liquid_sets_open(rho: np.ndarray, threshold: float):
    """Connected liquid sets (4-neighbour, rho > threshold) of a field
    rho[y, x] with plate rows and open (not periodic) x ends, largest first,
    each as [node count, centroid y, centroid x, reaches the row below the
    top plate, reaches the row above the bottom plate]."""
    ny, nx = rho.shape
    liq = rho > threshold
    liq[0] = liq[-1] = False
    lab, n = ndimage.label(liq)
    out = []
    for i in range(1, n + 1):
        ys, xs = np.nonzero(lab == i)
        out.append([int(ys.size), float(ys.mean()), float(xs.mean()), int(ys.max() == ny - 2),
                    int(ys.min() == 1)])
    out.sort(key=lambda r: -r[0])
    return out


def droplets(rho: np.ndarray, threshold: float):
    """Droplets touching each plate of a channel field rho[y, x] (plate rows
    included, periodic in x): connected sets (4-neighbour) of fluid nodes with
    rho > threshold that reach the first fluid row above the lower plate or
    below the upper plate.  Returns {"bottom": {count, mean_spacing},
    "top": {...}, "condensed_nodes": n}."""
    ny, nx = rho.shape
    liq = rho > threshold
    liq[0] = liq[-1] = False
    lab = _periodic_labels(liq)
    out = {}
    for name, row in (("bottom", 1), ("top", ny - 2)):
        ids = sorted(set(lab[row][lab[row] > 0].tolist()))
        centres = []
        for i in ids:
            cols = np.nonzero((lab == i).any(axis=0))[0]
            ang = 2 * np.pi * cols / nx
            c = (np.arctan2(np.sin(ang).mean(), np.cos(ang).mean()) % (2 * np.pi)) * nx / (2 * np.pi)
            centres.append(float(c))
        centres.sort()
        if len(centres) > 1:
            spacing = float(np.mean(np.diff(centres + [centres[0] + nx])))
        else:
            spacing = float(nx) if centres else 0.0
        out[name] = dict(count=len(ids), mean_spacing=spacing)
    out["condensed_nodes"] = int(liq.sum())
    return out


def field_differences(a, b, periodic_y: bool = False):
    """Per-field differences of run a from run b, each (rho, ux, uy, T):
    rho and T max relative, u max |du| / max |u_b| (u passes through 0)."""
    m = np.ones(a[0].shape, dtype=bool)
    if not periodic_y:
        m[0] = m[-1] = False
    e_rho = float(np.max(np.abs(a[0] - b[0])[m] / np.abs(b[0])[m]))
    e_T = float(np.max(np.abs(a[3] - b[3])[m] / np.abs(b[3])[m]))
    du = np.hypot(a[1] - b[1], a[2] - b[2])[m]
    um = float(np.hypot(b[1], b[2])[m].max())
    return dict(rho=e_rho, u=float(du.max() / um) if um > 0 else float(du.max()), T=e_T)


def equivalent_diameter(rho: np.ndarray, rho_l: float, rho_g: float) -> float:
    """Diameter of the disc holding the same liquid: area = sum of the liquid
    fraction (rho - rho_g)/(rho_l - rho_g) clipped to [0, 1], D = sqrt(4 A/pi)."""
    frac = np.clip((rho - rho_g) / (rho_l - rho_g), 0.0, 1.0)
    return float(np.sqrt(4.0 * frac.sum() / np.pi))


def d2_fit(t: np.ndarray, d2: np.ndarray):
    """Least-squares line d2 = a - K t; returns K and the coefficient of
    determination R^2."""
    A = np.column_stack([np.ones_like(t), -t])
    coef, *_ = np.linalg.lstsq(A, d2, rcond=None)
    pred = A @ coef
    ss_res = float(np.sum((d2 - pred) ** 2))
    ss_tot = float(np.sum((d2 - d2.mean()) ** 2))
    return float(coef[1]), 1.0 - ss_res / ss_tot if ss_tot > 0 else 1.0
