// Constants of the stencil-ELL matrix layout shared by the host setup and
// the residual kernel.
#pragma once

namespace dfmg {

// Slots of a row are stored in chunks of kEllVec consecutive values, so one
// lane reads a chunk with one vector load.
constexpr int kEllVec = 4;

// Subdomains with at most this many DOFs (the interior ones) are solved by
// one thread each in smoother variant 4; the others by one wavefront each.
constexpr int kSmallPatch = 8;

// Index maps with at most this many entries per row (the inverse subdomain
// maps, restriction and prolongation) are also stored in a fixed-width form:
// column w of row i at w * rows + i, unused slots -1, so a thread issues all
// of its index loads at once instead of walking a CSR row.  Wider maps keep
// only the CSR form.
constexpr int kEllMax = 24;

// Kernels are compiled for these fixed widths (a width is padded up to the
// next one); 0: the CSR form.
inline int ell_bucket(int w) { return w <= 0 ? 0 : (w <= 4 ? 4 : (w <= 8 ? 8 : (w <= 12 ? 12 : (w <= 24 ? 24 : 0)))); }

// Threads of a workgroup in the multiplicative sweep (one entry each; a
// subdomain's entries never straddle two workgroups); levels with a
// subdomain of more than kMultLanes DOFs use kMultLanesBig.
constexpr int kMultLanes = 256, kMultLanesBig = 1024;

// A lane of the wavefront that solves a boundary subdomain preloads this many
// coefficients of its row of the local inverse into registers.
constexpr int kBigRegs = 40;

}  // namespace dfmg
