"""Physics check of the peak list against the generator's truth (the paper's Fig. 1 analogue).

The paper compares the Hough transform with a chi^2 fit through the distributions and
resolutions of rho = sqrt(A^2 + B^2) and phi = tan^-1(B/A) (section 2). Its figure and dataset
are not available; this module makes the same comparison on synthetic events: track parameters
read out from the peaks (ht_readout) against the true circle centres, next to a least-squares
circle fit through the interaction point on each true track's hits.
"""
from __future__ import annotations

import math

import numpy as np

from . import synth


def lsq_circle_through_origin(x, y):
    """Centre (A, B) minimising sum (x^2 + y^2 - 2Ax - 2By)^2: the circle through the origin that
    best fits the hits, from the 2x2 normal equations."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    r2 = x * x + y * y
    m = np.array([[4 * np.dot(x, x), 4 * np.dot(x, y)], [4 * np.dot(x, y), 4 * np.dot(y, y)]])
    v = np.array([2 * np.dot(x, r2), 2 * np.dot(y, r2)])
    A, B = np.linalg.solve(m, v)
    return A, B


def wrap(d):
    return (d + math.pi) % (2 * math.pi) - math.pi


def evaluate(spec, tracks, ev, window: int = 1):
    """tracks: the readout of one event's peaks (structured array with a, b, t, A, B, rho, phi,
    theta, votes); ev: the synth.Event. A true track is in the acceptance when its centre lies
    inside the (A, B) range away from the edges and all 12 layers were hit; it is found when a
    peak lies within `window` bins of its centre bin in A and B and within one theta cell of its
    polar angle. Returns counts, efficiency, fake rate and resolutions."""
    dA = (spec.a_max - spec.a_min) / spec.n_a
    dB = (spec.b_max - spec.b_min) / spec.n_b
    tr = ev.truth
    n_tr = len(tr["A"])
    owner = ev.track_of_hit
    a_true = np.floor((tr["A"] - spec.a_min) / dA).astype(np.int64)
    b_true = np.floor((tr["B"] - spec.b_min) / dB).astype(np.int64)
    theta_true = 2 * np.arctan(np.exp(-tr["eta"]))
    t_true = np.floor(theta_true / (math.pi / spec.n_theta)).astype(np.int64)
    counts = np.bincount(owner[owner >= 0], minlength=n_tr)
    acc = ((a_true >= 1) & (a_true < spec.n_a - 1) & (b_true >= 1) & (b_true < spec.n_b - 1)
           & (counts == synth.LAYER_RADII_MM.size))
    used = np.zeros(len(tracks), bool)
    found, d_rho_ht, d_phi_ht, d_rho_fit, d_phi_fit = 0, [], [], [], []
    found_ids = []
    for k in np.flatnonzero(acc):
        m = ((np.abs(tracks["a"] - a_true[k]) <= window) & (np.abs(tracks["b"] - b_true[k]) <= window)
             & (np.abs(tracks["t"] - t_true[k]) <= 1))
        rho_t = math.hypot(tr["A"][k], tr["B"][k])
        phi_t = math.atan2(tr["B"][k], tr["A"][k])
        hx, hy = ev.x[owner == k], ev.y[owner == k]
        fa, fb = lsq_circle_through_origin(hx, hy)
        d_rho_fit.append((math.hypot(fa, fb) - rho_t) / rho_t)
        d_phi_fit.append(wrap(math.atan2(fb, fa) - phi_t))
        if not m.any():
            continue
        found += 1
        found_ids.append(int(k))
        used |= m
        best = np.flatnonzero(m)[np.argmax(tracks["votes"][m])]
        d_rho_ht.append((float(tracks["rho"][best]) - rho_t) / rho_t)
        d_phi_ht.append(wrap(float(tracks["phi"][best]) - phi_t))

    def rms(v):
        return float(np.sqrt(np.mean(np.square(v)))) if len(v) else None

    n_acc = int(acc.sum())
    return {"true_tracks": n_tr, "in_acceptance": n_acc, "found": found,
            "efficiency": found / n_acc if n_acc else None,
            "peaks": int(len(tracks)), "unmatched_peaks": int((~used).sum()),
            "fake_rate": float((~used).mean()) if len(tracks) else None,
            "rho_resolution_ht": rms(d_rho_ht), "phi_resolution_ht": rms(d_phi_ht),
            "rho_resolution_fit": rms(d_rho_fit), "phi_resolution_fit": rms(d_phi_fit),
            "bin_width_rel_rho": dA / 1000.0, "found_ids": found_ids,
            "acceptance_ids": [int(k) for k in np.flatnonzero(acc)]}
