// Batched elementwise combinations of the reverse sweep (host and device).
#pragma once

namespace fblts {

// One elementwise combination y = b*y + a0*x0 + a1*x1 + a2*x2 over
// [begin, end) (null inputs skipped), and a run of them for one launch.
struct LinDesc {
  double* y;
  const double* x0;
  const double* x1;
  const double* x2;
  double b, a0, a1, a2;
  int begin, end;
};
constexpr int kLinBatch = 24;
struct LinBatch {
  int n = 0, end_max = 0;
  LinDesc d[kLinBatch];
};

// Index ranges of the transposed tendency kernels for a cotangent supported
// on a prefix of the edges (Phi) or of the cells (Psi) of the region-
// contiguous numbering.  Every item past a kernel's range would add or store
// an exact zero, so the kernel stops there; the intermediates a later kernel
// reads past the range of the kernel that writes them are zeroed first, from
// that range's end to the z* bound.
struct VjpRange {
  int e1, c1, e2, v1, e3, c3, pe;   // Phi passes 1-6, and the edge records they read
  int zG, zR, zHD, zCDB, zBB, zQB, zHE, zZA, zHV;
};
struct PsiRange {
  int ne, nc, zT;                   // Psi edge and cell passes, and T's zero-fill bound
};

}  // namespace fblts
