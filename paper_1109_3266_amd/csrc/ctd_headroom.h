// Fixed-point headroom decision before a batch (plain C++, no HIP: the CPU
// tests compile it on its own).
//
// A batch of n histories whose photons start at <= e_max keV deposits at
// most b = n * e_max * 2^24 q in any voxel, so T_b <= b, and a voxel's sums
// after the batch are at most S1 + b and S2 + b^2.  The library keeps
// pessimistic bounds on the largest S1 and S2 of any voxel (the sum of the
// b and b^2 of every batch); only when those could pass 2^62 / 2^126 does it
// read back the exact per-voxel maxima the folds record, which admit the
// batch while S1 + b < 2^63 and S2 + b^2 < 2^128.
#pragma once

#include <cstdint>

namespace ctd {

enum HeadroomVerdict : int {
  kHeadroomOk = 0,        // admitted on the pessimistic bounds
  kHeadroomNeedExact = 1, // read the recorded maxima, then headroom_exact()
  kHeadroomBatch = 2,     // one batch alone could pass 2^62 q in a voxel
  kHeadroomOverflow = 3,  // the exact maxima leave no room
};

// First stage.  On kHeadroomOk, *s1 and *s2 receive the new bounds.
inline int headroom_bounds(double n, double e_max, double s1_bound, double s2_bound, double *s1,
                           double *s2) {
  const double b = n * e_max * 16777216.0;
  if (b >= 0x1p62) return kHeadroomBatch;
  *s1 = s1_bound + b;
  *s2 = s2_bound + b * b;
  if (*s1 >= 0x1p62 || *s2 >= 0x1p126) return kHeadroomNeedExact;
  return kHeadroomOk;
}

// Second stage, from the recorded maxima (largest S1, largest high word of
// S2).  On kHeadroomOk, *s1 and *s2 receive the new bounds.
inline int headroom_exact(double n, double e_max, uint64_t max_s1, uint64_t max_s2_hi,
                          double *s1, double *s2) {
  const double b = n * e_max * 16777216.0;
  *s1 = (double)max_s1 + b;
  *s2 = ((double)max_s2_hi + 1.0) * 0x1p64 + b * b;
  if (*s1 >= 0x1p63 || *s2 >= 0x1p128) return kHeadroomOverflow;
  return kHeadroomOk;
}

}  // namespace ctd
