"""Certification of FP32-mode moment differences against the FP64 oracle.

After one step from the same state, the GPU (FP32 particles) and the oracle
(FP64) hold slightly different particle states.  Their integer moments can
then differ only through particles whose deposit-deciding integers came out
differently: the cell, the quantised offset q = floor(o 2^b + 1/2) per axis
or the velocity code rint(v 2^s_v) per component.  A particle can flip one of
those only where its value lies within the FP32 rounding of the step of a
rounding boundary.

`certify_moments` finds every particle near such a boundary (a superset of
the flips: a particle whose integers agree contributes the same on both
sides), checks that each lies within rounding of its boundary, and asserts
that the moment difference is exactly the oracle's deposit of those
particles' GPU states minus their oracle states, for R, Gx, Gy and Gz
separately.  Every other node then agrees bit for bit.
"""

import numpy as np

from oracle import oracle as O

MARGIN = 1e-6   # in units of the quantisation step, beyond the two sides' spread


def by_id(d):
    o = np.argsort(d["id"], kind="stable")
    return {k: v[o] for k, v in d.items()}


def _straddles(a, b, half):
    """True where [min(a, b) - MARGIN, max(a, b) + MARGIN] contains a rounding
    boundary: an integer (half=False, floor) or a half-integer (half=True).
    The two values must lie less than one quantisation step apart (FP32
    rounding, not a different state), so a flip moves the integer by one."""
    assert np.all(np.abs(a - b) < 1.0), float(np.max(np.abs(a - b)))
    lo = np.minimum(a, b) - MARGIN
    hi = np.maximum(a, b) + MARGIN
    if half:
        lo, hi = lo - 0.5, hi - 0.5
    return np.floor(hi) != np.floor(lo)


def _deposit(p, species, st):
    o = O.Oracle(p)
    if len(st["id"]):
        o.set_particles(species, st["cell"], st["off"], st["v"], st["id"])
    o.step(O.DEPOSIT)
    return o.moments(species)


def certify_moments(p, species, pg, po, mg, mo, b, sv, max_fraction=0.5, columns=(0, 1, 2, 3)):
    """Asserts GPU moments mg equal the oracle moments mo up to certified
    rounding straddles, for the given moment columns (0 R, 1-3 G); returns
    (raw per-array relative differences, number of particles near a
    boundary).  The certified deposits are those at the particles'
    positions."""
    pg, po = by_id(pg), by_id(po)
    assert np.array_equal(pg["id"], po["id"])
    D = p["dim"]
    n = len(po["id"])
    near = np.zeros(n, dtype=bool)
    if n:
        cellmis = np.any(pg["cell"][:, :D] != po["cell"][:, :D], axis=1)
        near |= cellmis
        sc = float(2 ** b)
        same = ~cellmis   # a certified cell straddle has its offsets near 0 and 1
        for d in range(D):
            near[same] |= _straddles(pg["off"][same, d] * sc, po["off"][same, d] * sc, half=True)
        c = float(p.get("c_light", 0.0))

        def vel(u):
            if c > 0.0:
                return u / np.sqrt(1.0 + np.sum(u * u, axis=1, keepdims=True) / (c * c))
            return u

        vg, vo = vel(pg["v"]) * float(2 ** sv), vel(po["v"]) * float(2 ** sv)
        for k in range(3):
            near |= _straddles(vg[:, k], vo[:, k], half=True)
        assert near.sum() <= max(8, max_fraction * n), (near.sum(), n)
    sel = np.nonzero(near)[0]
    dg = _deposit(p, species, {k: v[sel] for k, v in pg.items()})
    do = _deposit(p, species, {k: v[sel] for k, v in po.items()})
    cols = list(columns)
    diff = mg.astype(np.int64) - mo.astype(np.int64)
    np.testing.assert_array_equal(diff[:, cols], (dg - do)[:, cols])
    raw = {}
    for m, name in enumerate(("R", "Gx", "Gy", "Gz")):
        den = float(np.max(np.abs(mo[:, m]))) if mo.size else 0.0
        raw[name] = float(np.max(np.abs(diff[:, m]))) / den if den > 0 else 0.0
    return raw, int(near.sum())
