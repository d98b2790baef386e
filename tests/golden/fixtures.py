"""Loaders for the paper's printed figure data (text fixtures in this folder)."""
from pathlib import Path

import numpy as np

HERE = Path(__file__).parent


def _rows(name):
    for line in (HERE / name).read_text().splitlines():
        if line and not line.startswith("#"):
            yield line.split()


def transmittance_dots():
    """{operator: [(tau_bar, T_bar)]} from Fig. 'Transmittance comparison'."""
    out = {}
    for o, x, y in _rows("fig_transmittance_dots.txt"):
        out.setdefault(o, []).append((float(x), float(y)))
    return out


def transmittance_mother():
    """{operator: array of T} sampled at tau_j = 2.02 j / 49, j = 0..49
    (printed with tau rounded to 4 decimals)."""
    out = {}
    for o, x, y in _rows("fig_transmittance_mother.txt"):
        out.setdefault(o, []).append(float(y))
    return {k: np.array(v) for k, v in out.items()}


def blending_concentric():
    """{operator: array [128, 5] of (x, red, green, blue, sum)} from
    Fig. 'Blending comparison' (a)."""
    out = {}
    for o, *vals in _rows("fig_blending_concentric.txt"):
        out.setdefault(o, []).append([float(v) for v in vals])
    return {k: np.array(v) for k, v in out.items()}
