// Control map of the optimal-perturbation ascent (the initial perturbation
// as the curl of a smooth vector potential), its adjoint, and the ascent
// update on the sphere of fixed initial perturbation energy.  The ascent
// itself is driven from the host: forward steps with checkpoints and the
// reverse sweep of tc_step_adjoint give the gradient of the final
// perturbation energy with respect to u^0, and these calls carry it to the
// control and take the step.
//
// Control layout: complex128 a[c][q][s][n], c = r, theta, z component of
// the vector potential, q = 0..3 the radial polynomial, (s, n) the stored
// mode.  Per mode (a = n k_theta, b = l k_z):
//   A_c(r) = sum_q a[c][q] B_q(r),  B_q = g T_q(xi),
//   g = 16 (r - r_i)^2 (r_o - r)^2,  xi = 2 (r - r_i) - 1,
//   u_r = i a A_z / r - i b A_theta,  u_theta = i b A_r - d_r A_z,
//   u_z = d_r A_theta + A_theta / r - i a A_r / r,
// with d_r A_c from the polynomials' exact derivatives.  Mode (0,0) and the
// empty axial slot are not controls.
#include <algorithm>
#include <cmath>

#include "tc_internal.h"

namespace tc {

namespace {

__device__ __forceinline__ cd cz() { return cd{0.0, 0.0}; }
__device__ __forceinline__ cd cadd2(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd cscl(cd v, double w) { return cd{v.x * w, v.y * w}; }
__device__ __forceinline__ cd ciw(cd v, double w) { return cd{-w * v.y, w * v.x}; }  // i w v
__device__ __forceinline__ cd cconj2(cd v) { return cd{v.x, -v.y}; }

// B_q(r) and d_r B_q(r), q = 0..3
__device__ __forceinline__ void radial_basis(double r, double ri, double ro, double (&B)[4], double (&dB)[4]) {
  const double xi = 2.0 * (r - ri) - 1.0;
  const double T[4] = {1.0, xi, 2.0 * xi * xi - 1.0, 4.0 * xi * xi * xi - 3.0 * xi};
  const double dT[4] = {0.0, 2.0, 8.0 * xi, 2.0 * (12.0 * xi * xi - 3.0)};
  const double x = r - ri, y = ro - r;
  const double g = 16.0 * x * x * y * y;
  const double dg = 32.0 * x * y * y - 32.0 * x * x * y;
  for (int q = 0; q < 4; ++q) {
    B[q] = g * T[q];
    dB[q] = dg * T[q] + g * dT[q];
  }
}

__device__ __forceinline__ bool is_control(const Dims& d, int s, int n) { return s != d.nyq && !(s == 0 && n == 0); }

}  // namespace

// u = U_c + B a, one thread per (node, slot).
__global__ void k_control_velocity(const double* __restrict__ rc, Dims d, double ri, double ro, double C1, double C2,
                                   const cd* __restrict__ a, cd* __restrict__ u) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.F) return;
  const int j = (int)(idx / d.S);
  const int64_t sn = idx - (int64_t)j * d.S;
  const int s = (int)(sn / d.mt), n = (int)(sn - (int64_t)s * d.mt);
  const double r = rc[(int64_t)j * RC_N + RC_R], ir = rc[(int64_t)j * RC_N + RC_IR];
  cd up = cz(), um = cz(), uz = cz();
  if (is_control(d, s, n)) {
    double B[4], dB[4];
    radial_basis(r, ri, ro, B, dB);
    cd A[3], dA[3];
    for (int c = 0; c < 3; ++c) {
      A[c] = dA[c] = cz();
      for (int q = 0; q < 4; ++q) {
        const cd v = a[((int64_t)(c * 4 + q) * d.mz + s) * d.mt + n];
        A[c] = cadd2(A[c], cscl(v, B[q]));
        dA[c] = cadd2(dA[c], cscl(v, dB[q]));
      }
    }
    const double an = n * d.kt, bl = (s < d.half ? s : s - d.mz) * d.kz;
    const cd ur = cadd2(ciw(A[2], an * ir), ciw(A[1], -bl));
    const cd ut = cadd2(ciw(A[0], bl), cscl(dA[2], -1.0));
    uz = cadd2(cadd2(dA[1], cscl(A[1], ir)), ciw(A[0], -an * ir));
    const cd iut = ciw(ut, 1.0);
    up = cadd2(ur, iut);
    um = cd{ur.x - iut.x, ur.y - iut.y};
  } else if (s == 0 && n == 0) {
    const double U = C1 * r + C2 / r;  // circular Couette flow, u+- = +-i U
    up = cd{0.0, U};
    um = cd{0.0, -U};
  }
  u[idx] = up;
  u[d.F + idx] = um;
  u[2 * d.F + idx] = uz;
}

// g_a = B^H g (before the Hermitian projection), one thread per slot
// marching through the nodes.
__global__ void k_control_gradient(const double* __restrict__ rc, Dims d, double ri, double ro,
                                   const cd* __restrict__ g, cd* __restrict__ ga) {
  const int64_t sn = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sn >= d.S) return;
  const int s = (int)(sn / d.mt), n = (int)(sn - (int64_t)s * d.mt);
  cd acc[3][4];
  for (int c = 0; c < 3; ++c)
    for (int q = 0; q < 4; ++q) acc[c][q] = cz();
  if (is_control(d, s, n)) {
    const double an = n * d.kt, bl = (s < d.half ? s : s - d.mz) * d.kz;
    for (int j = 0; j < d.n_r; ++j) {
      const double r = rc[(int64_t)j * RC_N + RC_R], ir = rc[(int64_t)j * RC_N + RC_IR];
      const int64_t o = (int64_t)j * d.S + sn;
      const cd gp = g[o], gm = g[d.F + o], gz = g[2 * d.F + o];
      const cd gr = cadd2(gp, gm);
      const cd gt = ciw(cd{gp.x - gm.x, gp.y - gm.y}, -1.0);
      // cotangents of A_c and d_r A_c
      const cd GA[3] = {cadd2(ciw(gt, -bl), ciw(gz, an * ir)), cadd2(ciw(gr, bl), cscl(gz, ir)), ciw(gr, -an * ir)};
      const cd GdA[3] = {cz(), gz, cscl(gt, -1.0)};
      double B[4], dB[4];
      radial_basis(r, ri, ro, B, dB);
      for (int c = 0; c < 3; ++c)
        for (int q = 0; q < 4; ++q) acc[c][q] = cadd2(acc[c][q], cadd2(cscl(GA[c], B[q]), cscl(GdA[c], dB[q])));
    }
  }
  for (int c = 0; c < 3; ++c)
    for (int q = 0; q < 4; ++q) ga[((int64_t)(c * 4 + q) * d.mz + s) * d.mt + n] = acc[c][q];
}

// Orthogonal projection on controls with x(-l, 0) = conj(x(l, 0)): one
// thread per (c, q, l), 1 <= l < m_z/2.
__global__ void k_control_hermitian(Dims d, cd* __restrict__ x) {
  const int h = d.mz / 2;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 12 * (h - 1)) return;
  const int cq = idx / (h - 1), l = 1 + idx % (h - 1);
  cd* col = x + (int64_t)cq * d.mz * d.mt;
  const cd p = col[(int64_t)l * d.mt], m = col[(int64_t)(d.mz - l) * d.mt];
  const cd avg = cscl(cadd2(p, cconj2(m)), 0.5);
  col[(int64_t)l * d.mt] = avg;
  col[(int64_t)(d.mz - l) * d.mt] = cconj2(avg);
}

// Block partial sums of <x, y>, <y, y> and <x, x> (controls; Re(conj(x) y)).
__global__ void k_control_dots(int64_t count, const cd* __restrict__ x, const cd* __restrict__ y,
                               double* __restrict__ part) {
  __shared__ double red[3][256];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const cd u = x[i], v = y[i];
    a += u.x * v.x + u.y * v.y;
    b += v.x * v.x + v.y * v.y;
    c += u.x * u.x + u.y * u.y;
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) part[3 * blockIdx.x + k] = red[k][0];
}

// out = s (a + tau (gJ - beta gE)), on the controls only (zero elsewhere).
// (a and out may be the same array)
__global__ void k_control_axpy(Dims d, int64_t count, const cd* a, const cd* __restrict__ gJ,
                               const cd* __restrict__ gE, double tau, double beta, double s, cd* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t sn = i % d.S;
  const int sl = (int)(sn / d.mt), n = (int)(sn - (int64_t)sl * d.mt);
  cd v = cz();
  if (is_control(d, sl, n)) {
    const cd x = a[i];
    const cd p = gJ ? cd{gJ[i].x - beta * gE[i].x, gJ[i].y - beta * gE[i].y} : cz();
    v = cd{s * (x.x + tau * p.x), s * (x.y + tau * p.y)};
  }
  out[i] = v;
}

}  // namespace tc

using namespace tc;

namespace {

constexpr int DOT_BLOCKS = 512;

void couette_constants(const tc_ctx* c, double& C1, double& C2) {
  const double eta = c->eta, Ri = c->d.Re_i, Ro = c->d.Re_o;
  C1 = (Ro - eta * Ri) / (1.0 + eta);
  C2 = eta * (Ri - eta * Ro) / ((1.0 - eta) * (1.0 - eta * eta));
}

hipError_t control_velocity(tc_ctx* c, const cd* a, cd* u, bool with_couette) {
  double C1, C2;
  couette_constants(c, C1, C2);
  if (!with_couette) C1 = C2 = 0.0;
  const unsigned blocks = (unsigned)((c->d.F + 255) / 256);
  hipLaunchKernelGGL(k_control_velocity, dim3(blocks), dim3(256), 0, c->stream, c->rc_dev, c->d, c->r_i, c->r_o, C1,
                     C2, a, u);
  return hipGetLastError();
}

// Host-side sums of <x, y>, <y, y>, <x, x> (synchronous).
hipError_t control_dots(tc_ctx* c, const cd* x, const cd* y, double& xy, double& yy, double& xx) {
  const int64_t count = 12 * c->d.S;
  hipLaunchKernelGGL(k_control_dots, dim3(DOT_BLOCKS), dim3(256), 0, c->stream, count, x, y, c->red);
  hipError_t e = hipGetLastError();
  double h[3 * DOT_BLOCKS];
  if (e == hipSuccess) e = hipMemcpyAsync(h, c->red, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  xy = yy = xx = 0.0;
  for (int b = 0; b < DOT_BLOCKS; ++b) {
    xy += h[3 * b];
    yy += h[3 * b + 1];
    xx += h[3 * b + 2];
  }
  return e;
}

}  // namespace

extern "C" {

tc_status tc_control_velocity(tc_ctx* c, const void* a, void* u) {
  if (!c) return TC_EINVAL;
  if (!a || !u) return fail(c, TC_EINVAL, "NULL array");
  return hip_check(c, control_velocity(c, static_cast<const cd*>(a), static_cast<cd*>(u), true),
                   "tc_control_velocity");
}

tc_status tc_control_gradient(tc_ctx* c, const void* g, void* ga) {
  if (!c) return TC_EINVAL;
  if (!g || !ga) return fail(c, TC_EINVAL, "NULL array");
  const Dims& d = c->d;
  hipLaunchKernelGGL(k_control_gradient, dim3((unsigned)((d.S + 63) / 64)), dim3(64), 0, c->stream, c->rc_dev, d,
                     c->r_i, c->r_o, static_cast<const cd*>(g), static_cast<cd*>(ga));
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && d.half > 1) {
    hipLaunchKernelGGL(k_control_hermitian, dim3((unsigned)((12 * (d.half - 1) + 255) / 256)), dim3(256), 0,
                       c->stream, d, static_cast<cd*>(ga));
    e = hipGetLastError();
  }
  return hip_check(c, e, "tc_control_gradient");
}

tc_status tc_control_ascent_update(tc_ctx* c, const void* a, const void* gJ, const void* gE, double tau, double E0,
                                   void* a_out, double* stats) {
  if (!c) return TC_EINVAL;
  if (!a || !a_out || ((gJ == nullptr) != (gE == nullptr))) return fail(c, TC_EINVAL, "NULL array");
  if (!(E0 > 0.0) || !std::isfinite(tau)) return fail(c, TC_EINVAL, "E0 must be positive and tau finite");
  const Dims& d = c->d;
  const int64_t count = 12 * d.S;
  const cd* A = static_cast<const cd*>(a);
  const cd* GJ = static_cast<const cd*>(gJ);
  const cd* GE = static_cast<const cd*>(gE);
  cd* out = static_cast<cd*>(a_out);
  double jE = 0.0, EE = 1.0, JJ = 0.0, aa = 0.0, d0 = 0.0, d1 = 0.0;
  hipError_t e = control_dots(c, A, A, d0, d1, aa);
  if (e == hipSuccess && GJ) e = control_dots(c, GJ, GE, jE, EE, JJ);
  if (e != hipSuccess) return hip_check(c, e, "tc_control_ascent_update");
  if (GJ && !(EE > 0.0)) return fail(c, TC_EINVAL, "the energy gradient is zero");
  const double beta = jE / EE;
  // |p|^2 = |gJ|^2 - <gJ, gE>^2 / |gE|^2
  const double pp = GJ ? std::max(0.0, JJ - jE * beta) : 0.0;
  const unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(k_control_axpy, dim3(blocks), dim3(256), 0, c->stream, d, count, A, GJ, GE, tau, beta, 1.0, out);
  e = hipGetLastError();
  // energy of the new perturbation (the curl work buffer holds B out)
  c->omega_fresh = false;
  if (e == hipSuccess) e = control_velocity(c, out, c->omega, false);
  double E = 0.0;
  if (e == hipSuccess) e = energy_of(c, c->omega, E);
  if (e != hipSuccess) return hip_check(c, e, "tc_control_ascent_update");
  if (!(E > 0.0)) return fail(c, TC_EINVAL, "the updated control has no energy");
  const double s = std::sqrt(E0 / E);
  hipLaunchKernelGGL(k_control_axpy, dim3(blocks), dim3(256), 0, c->stream, d, count, out, nullptr, nullptr, 0.0, 0.0,
                     s, out);
  e = hipGetLastError();
  if (stats) {
    stats[0] = beta;
    stats[1] = E;
    stats[2] = s;
    stats[3] = std::sqrt(pp);
    stats[4] = std::sqrt(aa);
  }
  return hip_check(c, e, "tc_control_ascent_update");
}

}  // extern "C"
