"""Comparison of a GPU space-time solution with the stored oracle data of
tests/golden/<config>_samples.json (written by tests/golden/make_golden.py from
the CPU oracle only).

Bar: the paper's stopping tolerance, a relative error of 1e-10 in the discrete
L^inf(0,T; L^2) norm (Section 5).  With B = 1e-10 max_n ||u_n^ref||_2 an error
within the bar satisfies, at every level n,
  * | ||u_n||_2 - ||u_n^ref||_2 | <= ||e_n||_2 <= B            (triangle inequality)
  * |e_n(x)| <= ||e_n||_2 <= B at every point x
  * <w, e_n> ~ N(0, ||e_n||^2) for a standard-normal weight array w drawn
    independently of the error, so |<w, e_n>| <= 6 B except with probability
    2e-9 per projection (six standard deviations)
and the discrete mass and energy of every level match the oracle's.
"""
from __future__ import annotations

import json
import os

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name: str) -> dict:
    with open(os.path.join(GOLDEN_DIR, f"{name}_samples.json")) as f:
        return json.load(f)


def weights(g: dict, shape):
    seed = g["proj_seed"]
    return [np.random.default_rng(seed + q).standard_normal(shape) for q in range(len(g["projections"][0]))]


def compare(U: np.ndarray, g: dict) -> dict:
    """Deviations of U ([N_t][N][N] FP64, host) from the stored oracle data,
    each divided by max_n ||u_n^ref||_2.  Returns a dict of the largest
    relative deviation per kind and their maximum ('rel')."""
    nt = U.shape[0]
    nref = np.asarray(g["norms"])
    scale = float(np.max(nref))
    flat = U.reshape(nt, -1)
    norms = np.sqrt(np.sum(flat * flat, axis=1))
    d_norm = float(np.max(np.abs(norms - nref))) / scale
    ws = weights(g, U.shape[1:])
    proj = np.array([[float(np.sum(w * U[n])) for w in ws] for n in range(nt)])
    d_proj = float(np.max(np.abs(proj - np.asarray(g["projections"])))) / scale
    pts = np.asarray(g["points"])
    d_pt = 0.0
    for lev, vals in g["samples"].items():
        got = U[int(lev) - 1][pts[:, 0], pts[:, 1]]
        d_pt = max(d_pt, float(np.max(np.abs(got - np.asarray(vals)))))
    d_pt /= scale
    return {"norms": d_norm, "projections": d_proj, "points": d_pt, "rel": max(d_norm, d_proj / 6.0, d_pt)}


def assert_within(U: np.ndarray, g: dict, tol: float = 1e-10) -> dict:
    c = compare(U, g)
    assert c["norms"] <= tol, c
    assert c["points"] <= tol, c
    assert c["projections"] <= 6.0 * tol, c
    return c
