"""CPU oracle for super-droplet displacement and cell re-segmentation.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests, the smoke
check and the CPU-baseline leg of the benchmark may call it; the product path
never does.  Plain numpy, IEEE fp64, no fused multiply-add (numpy does not
contract), written from the method, not from any listing.

The PySDM v1 paper lists particle displacement among the dynamics other than
coalescence (section "API in brief") and couples the particles to a prescribed
2D single-eddy flow in its kinematic examples (section "Kinematic
(prescribed-flow) examples"), but gives no scheme.  Readings taken here:

  - the domain is nx x nz cells, cell index c = ix * nz + iz, periodic in both
    directions; along an axis of one cell a droplet that crosses a face
    re-enters the same cell (its shift is 0), and along an axis of two cells
    both directions lead to the other cell (its shift is taken as +1), so a
    1D column (nx = 1) is a grid like any other;
  - a super-droplet carries its position inside its cell as two fractions
    (wx, wz) in [0, 1);
  - the flow is given as Courant numbers on cell faces (a staggered grid):
    cx[ix, iz] on the face between cells ix - 1 and ix (shape (nx + 1, nz)),
    cz[ix, iz] on the face between cells iz - 1 and iz (shape (nx, nz + 1));
  - one explicit first-order step: the displacement along each axis is the
    Courant number interpolated linearly between the cell's two faces at the
    droplet's position, d = (1 - w) * c_low + w * c_high, evaluated as two
    products and one sum in that order; then w' = w + d;
  - the cell shift is floor(w'), the new fraction w' - floor(w'); a fraction
    that rounds to 1 (only possible for tiny negative w') becomes 0 in the
    next cell up;
  - |d| < 1 is required (Courant condition), and positions are fractions in
    [0, 1).  A droplet with |d| >= 1 (or not finite), or whose fraction is out
    of range, raises the COURANT flag; its shift is then clamped to [-1, 1]
    (the result is not meaningful, only defined);
  - re-segmentation is a stable sort of the slots by their new cell: slots of
    one new cell keep their old order (old cell, then old slot), which is the
    order the coalescence step's per-slot random numbers are tied to.  Every
    slot moves, including those with multiplicity 0.
"""
from __future__ import annotations

import numpy as np

ST_COURANT = 1


def axis_step(w, c_low, c_high):
    """New fraction, cell shift and Courant-violation mask along one axis."""
    w = np.asarray(w, dtype=np.float64)
    d = (1.0 - w) * c_low + w * c_high
    bad = ~(np.abs(d) < 1.0) | ~((w >= 0.0) & (w < 1.0))
    wn = w + d
    f = np.floor(wn)
    frac = wn - f
    up = frac >= 1.0
    frac = np.where(up, 0.0, frac)
    s = f + up.astype(np.float64)
    # clamp to one cell (only reached under the flag); a NaN counts as -1
    shift = np.where(np.isnan(s), -1.0, np.clip(s, -1.0, 1.0)).astype(np.int64)
    return frac, shift, bad


def cell_coords(cell_off, nz):
    """(ix, iz) of every slot from the cell offsets."""
    counts = np.diff(np.asarray(cell_off, dtype=np.int64))
    c = np.repeat(np.arange(counts.size, dtype=np.int64), counts)
    return c // nz, c % nz


def periodic_shift(shift, n_axis):
    """The shift along an axis of n_axis cells: 0 if the axis has one cell,
    +1 for any move if it has two (both neighbours are the same cell)."""
    if n_axis == 1:
        return np.zeros_like(shift)
    if n_axis == 2:
        return (shift != 0).astype(shift.dtype)
    return shift


def displace(nx, nz, cx, cz, pos, cell_off):
    """One displacement step.  pos: (2, n) fractions (x row, z row).

    Returns (new_pos, new_cell, flags): new_pos (2, n) in the old slot order,
    new_cell (n,) the destination cell of every slot, flags the status word.
    """
    cx = np.asarray(cx, dtype=np.float64)
    cz = np.asarray(cz, dtype=np.float64)
    assert cx.shape == (nx + 1, nz) and cz.shape == (nx, nz + 1)
    ix, iz = cell_coords(cell_off, nz)
    wx, sx, bx = axis_step(pos[0], cx[ix, iz], cx[ix + 1, iz])
    wz, sz, bz = axis_step(pos[1], cz[ix, iz], cz[ix, iz + 1])
    sx = periodic_shift(sx, nx)
    sz = periodic_shift(sz, nz)
    jx = (ix + sx) % nx
    jz = (iz + sz) % nz
    flags = ST_COURANT if (bx.any() or bz.any()) else 0
    return np.stack([wx, wz]), jx * nz + jz, flags


def resegment(new_cell, n_cells):
    """Stable order of the slots by new cell, and the new cell offsets."""
    order = np.argsort(new_cell, kind="stable")
    off = np.zeros(n_cells + 1, dtype=np.int64)
    off[1:] = np.cumsum(np.bincount(new_cell, minlength=n_cells))
    return order, off


def displace_resegment(nx, nz, cx, cz, xi, v, attrs, pos, cell_off):
    """Displacement followed by re-segmentation: the whole state in the new
    slot order.  Returns (xi, v, attrs, pos, cell_off, flags)."""
    new_pos, new_cell, flags = displace(nx, nz, cx, cz, pos, cell_off)
    order, off = resegment(new_cell, nx * nz)
    attrs = np.asarray(attrs)
    return (np.asarray(xi)[order], np.asarray(v)[order], attrs[:, order], new_pos[:, order], off,
            flags)
