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

}  // namespace fblts
