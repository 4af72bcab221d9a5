// Work units over particle bounding boxes, shared by the MEM remap (binary
// mapping, links, uncovered cells; Sec. 2.2) and the PSM list stages (solid
// fractions and overlap pairs; Sec. 2.3.2).  A particle's box starts at
// floor(X - R - 2) per axis; the slot grid is `side` cells wide for the
// largest particle, and a unit is a row range of one slab of it.
#pragma once

#include "common.h"

namespace lbm {

// Cells per axis of particle p's own box: ceil(D) + 6 cells reach R + 3 beyond
// the centre, past every solid, cut or uncovered cell and every link of p and
// past the cells p uncovered in its previous remap (it moves less than one
// cell per rigid-body step).
__device__ __forceinline__ int bbox_extent(const PartDev& P, int p, int side) {
  return min(side, (int)ceil(P.D[p]) + 6);
}

// Cells of unit U inside the own box: rows [U.y0, min(U.y1, ext)) of ext cells
// of slab U.z < ext.  Every stage visits exactly these, in this order, so
// counts and scanned offsets agree between stages.
__device__ __forceinline__ int unit_cells(const Unit& U, int ext) {
  const int y1 = min(U.y1, ext);
  return (U.z < ext && y1 > U.y0) ? (y1 - U.y0) * ext : 0;
}

// i in [-n, 2n) wrapped into [0, n).  Box cells qualify: the box corner is
// above -n and the box (at most min(nx, ny, nz) wide) ends below 2n; so do
// their lattice neighbours.
__device__ __forceinline__ int wrap_near(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

// The cells c = a .. b-1 of a unit (row length ext, first row y0), with row dy
// and column dx carried along instead of divided out per cell.
#define BBOX_FOR_CELLS(c, a, b, y0, ext, dy, dx)                                  \
  for (int c = (a), dy = (y0) + (a) / (ext), dx = (a) % (ext); c < (b);           \
       ++c, (++dx == (ext) ? (dx = 0, ++dy) : 0))

// The cells c = a, a + s, a + 2s, ... below b, with qs = s / ext, rs = s % ext.
#define BBOX_FOR_CELLS_STRIDED(c, a, b, s, qs, rs, y0, ext, dy, dx)               \
  for (int c = (a), dy = (y0) + (a) / (ext), dx = (a) % (ext); c < (b);           \
       c += (s), dx += (rs), dy += (qs), (dx >= (ext) ? (dx -= (ext), ++dy) : 0))

}  // namespace lbm
