"""Element-wise parity measures shared by the GPU tests (test infrastructure; no method arithmetic).

nmse: ||got - ref||^2 / ||ref||^2 over the whole result.
line_errors: the largest relative error of any single line along each of two axes (by default the
last two: a k-space row or column of one coil, or of one echo and coil): ||got_line - ref_line|| / ||ref_line||,
with the denominator floored at `floor` times the root-mean-square line norm so that lines carrying
almost no signal (the far edge of k-space) are judged against the result's scale.  A percent-level
error confined to one lifted line or one k-space line shows up here although it would vanish in the
NMSE of the whole result.
"""

import numpy as np


def nmse(got, ref):
    return float(np.sum(np.abs(got - ref) ** 2) / np.sum(np.abs(ref) ** 2))


def line_errors(got, ref, floor=1e-3, axes=(-1, -2)):
    d = np.asarray(got) - np.asarray(ref)
    out = {}
    for ax, name in zip(axes, ("rows", "cols")):
        num = np.sqrt(np.sum(np.abs(d) ** 2, axis=ax))
        den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=ax))
        fl = floor * np.sqrt(np.mean(den ** 2))
        out[name] = float(np.max(num / np.maximum(den, fl)))
    return out


def check(got, ref, nmse_bar, line_bar, label="", axes=(-1, -2)):
    """Assert NMSE < nmse_bar and every line's relative error < line_bar (lines along the two given
    axes); print the measured levels."""
    e = nmse(got, ref)
    le = line_errors(got, ref, axes=axes)
    print(f"{label}: nmse={e:.3e} line rel err rows={le['rows']:.3e} cols={le['cols']:.3e}", flush=True)
    assert e < nmse_bar, (label, e)
    assert max(le.values()) < line_bar, (label, le)
    return e, le
