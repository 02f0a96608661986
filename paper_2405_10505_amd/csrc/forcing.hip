// gfx950 kernels for the cyclone wind forcing of the wind-stress term
// (paper eq. hurricane_model: the stress uses the 10 m wind u_W at edges).
//
// The wind is an analytic Holland (1980) gradient-wind vortex whose centre
// moves along a great circle of the sphere at constant speed.  It is evaluated
// once per coarse step, before the step's first stage, at model time
// t = t0 + k dt where k counts the coarse steps since the storms were set (a
// solver: its latest storm; an ensemble: its first).  k lives in device memory
// (advanced by a one-thread tick kernel at the end of the step) so that a
// captured step graph replays with the storm moving.
//
// Per edge: great-circle distance to the centre r = R atan2(|x cross c|, x.c),
// V(r) = sqrt((B/rho_a)(Rm/r)^B dp exp(-(Rm/r)^B) + (r f/2)^2) - r|f|/2 with
// f = 2 Omega z, swirl sign(f_c) V (x cross r_hat) (counter-clockwise about the
// centre in the northern hemisphere; r_hat points away from the centre) plus a
// translation part v_trans (V / V(Rm, f_c)) along the track direction projected
// onto the tangent plane.  Outputs W.n_e and W.t_e with t_e = x cross n_e,
// and the wind-stress coefficient of the forcing at the edge,
// C_W = (rho_air / rho_water)(0.75 + 0.067 |W|) 1e-3 (Garratt's 10 m drag law
// in kinematic form; |W| from the two tangent-plane components).
//
// Members are innermost (item = edge * nm + member), each member with its
// own storm parameters, or calm air (zero wind) without a storm.
//
// Bytes per edge: 6 doubles read (unit position, unit normal), 3 per member written.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fblts_internal.h"

namespace fblts {

namespace {

struct V3 {
  double x, y, z;
};
__device__ __forceinline__ V3 v3(double a, double b, double c) { return V3{a, b, c}; }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ V3 axpy(double s, V3 a, V3 b) { return v3(s * a.x + b.x, s * a.y + b.y, s * a.z + b.z); }
__device__ __forceinline__ V3 scale(double s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ double norm(V3 a) { return sqrt(dot(a, a)); }

// Holland gradient-wind speed at distance r (m) and Coriolis parameter f.
__device__ __forceinline__ double holland_speed(const CycloneParams& a, double r, double f) {
  r = fmax(r, 1.0);
  const double s = pow(a.rm / r, a.b);
  const double rf2 = 0.5 * r * f;
  return sqrt(a.b / a.rho_air * s * a.dp * exp(-s) + rf2 * rf2) - 0.5 * r * fabs(f);
}

__device__ __forceinline__ double wind_coefficient(double rho_ratio, double wn, double wt) {
  return rho_ratio * (0.75 + 0.067 * sqrt(wn * wn + wt * wt)) * 1e-3;
}

__global__ void __launch_bounds__(kBlock) k_cyclone(CycloneArgs a) {
  const long item = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= ((long)a.E << a.nm_log2)) return;
  const int e = (int)(item >> a.nm_log2);
  const CycloneParams& P = a.p[item & ((1 << a.nm_log2) - 1)];
  if (!P.enabled) {
    a.wn[item] = 0.0;
    a.wt[item] = 0.0;
    a.wc[item] = wind_coefficient(a.rho_ratio, 0.0, 0.0);
    return;
  }
  // storm centre at this step: c0 rotated about the track axis
  const double t = (double)a.clock[0] * a.dt;
  const double ang = P.omega_track * (t + P.t0);
  const double ca = cos(ang), sa = sin(ang);
  const V3 c0 = v3(P.c0[0], P.c0[1], P.c0[2]);
  const V3 k = v3(P.axis[0], P.axis[1], P.axis[2]);
  const V3 kc = cross(k, c0);
  const double kdc = dot(k, c0);
  const V3 c = v3(c0.x * ca + kc.x * sa + k.x * kdc * (1.0 - ca), c0.y * ca + kc.y * sa + k.y * kdc * (1.0 - ca),
                  c0.z * ca + kc.z * sa + k.z * kdc * (1.0 - ca));
  const V3 x = v3(a.x[e], a.x[a.E + e], a.x[2 * a.E + e]);
  const V3 n = v3(a.n[e], a.n[a.E + e], a.n[2 * a.E + e]);

  const double cosang = dot(x, c);
  const double sinang = norm(cross(x, c));
  const double r = P.radius * atan2(sinang, cosang);
  const double f = 2.0 * P.omega * x.z;
  const double fc = 2.0 * P.omega * c.z;
  const double V = holland_speed(P, r, f);
  const double vmax = holland_speed(P, P.rm, fc);

  const V3 ct = axpy(-cosang, x, c);  // towards the centre, in the tangent plane at x
  const double nrm = norm(ct);
  const V3 rhat = nrm > 0.0 ? scale(-1.0 / nrm, ct) : v3(0.0, 0.0, 0.0);
  const V3 sw = scale(fc >= 0.0 ? V : -V, cross(x, rhat));
  const V3 tau = cross(k, c);
  const V3 tx = axpy(-dot(x, tau), x, tau);
  const V3 th = scale(1.0 / fmax(norm(tx), 1e-300), tx);
  const V3 W = axpy(vmax > 0.0 ? P.v_trans * V / vmax : 0.0, th, sw);

  const double wn = dot(W, n), wt = dot(W, cross(x, n));
  a.wn[item] = wn;
  a.wt[item] = wt;
  a.wc[item] = wind_coefficient(a.rho_ratio, wn, wt);
}

__global__ void k_clock_tick(long long* clock) {
  if (blockIdx.x == 0 && threadIdx.x == 0) clock[0] = clock[0] + 1;
}

}  // namespace

void launch_cyclone(const CycloneArgs& a, hipStream_t st) {
  const long items = (long)a.E << a.nm_log2;
  if (items <= 0) return;
  hipLaunchKernelGGL(k_cyclone, dim3((unsigned)((items + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, a);
}

void launch_clock_tick(long long* clock, hipStream_t st) {
  hipLaunchKernelGGL(k_clock_tick, dim3(1), dim3(64), 0, st, clock);
}

}  // namespace fblts
