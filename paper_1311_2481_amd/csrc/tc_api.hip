// C-ABI entry points of libtc: context set-up (radial grid, FD weights,
// factorisation), state handling, the time-step driver and diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "tc_internal.h"

using namespace tc;

namespace tc {

tc_status fail(tc_ctx* c, tc_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

tc_status hip_check(tc_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return TC_OK;
  return fail(c, TC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

void timer_begin(tc_ctx* c, int which) {
  if (!c->timing) return;
  KernelTimer& t = c->timers[which];
  t.open = false;
  if ((size_t)(t.used + 2) > t.ev.size()) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      if (a) (void)hipEventDestroy(a);
      (void)hipGetLastError();
      return;  // this launch goes untimed
    }
    t.ev.push_back(a);
    t.ev.push_back(b);
  }
  if (hipEventRecord(t.ev[t.used], c->stream) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  t.open = true;
}

void timer_end(tc_ctx* c, int which) {
  if (!c->timing) return;
  KernelTimer& t = c->timers[which];
  if (!t.open) return;
  t.open = false;
  if (hipEventRecord(t.ev[t.used + 1], c->stream) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  t.used += 2;
}

}  // namespace tc

namespace {

thread_local std::string g_init_error;

// ---------------------------------------------------------------- radial grid
// Nodes of eq. nodeDist with j = 0..M:  r_j = (1+eta)/(2(1-eta)) +
// asin(-alpha cos(pi j / M)) / (2 asin alpha), alpha -> 0 the Chebyshev
// limit.  -cos(pi j/M) is evaluated as sin(pi (j - M/2) / M), exact at the
// walls and odd about mid-gap.
std::vector<double> radial_nodes(int n_r, double eta, double alpha) {
  std::vector<double> r(n_r);
  const int M = n_r - 1;
  const long double centre = (1.0L + eta) / (2.0L * (1.0L - eta));
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < n_r; ++j) {
    const long double x = std::sin(pi * ((long double)j - 0.5L * M) / (long double)M);
    long double v;
    if (alpha == 0.0)
      v = centre + 0.5L * x;
    else
      v = centre + std::asin((long double)alpha * x) / (2.0L * std::asin((long double)alpha));
    r[j] = (double)v;
  }
  return r;
}

// Finite-difference weights by Fornberg's recursion (Math. Comp. 51, 1988):
// delta[m][k][v] is the weight of node v for the m-th derivative using
// nodes 0..k; built up one node at a time.  Returns weights for m = 1, 2
// at z from the nodes x[0..n-1].
void fd_weights(double z, const double* x, int n, double* w1, double* w2) {
  const int MD = 2;
  std::vector<long double> delta((size_t)(MD + 1) * n * n, 0.0L);
  auto D = [&](int m, int k, int v) -> long double& { return delta[((size_t)m * n + k) * n + v]; };
  D(0, 0, 0) = 1.0L;
  long double c1 = 1.0L;
  for (int k = 1; k < n; ++k) {
    long double c2 = 1.0L;
    for (int v = 0; v < k; ++v) {
      const long double c3 = (long double)x[k] - x[v];
      c2 *= c3;
      for (int m = 0; m <= std::min(k, MD); ++m) {
        const long double prev = D(m, k - 1, v);
        const long double prevm = m > 0 ? D(m - 1, k - 1, v) : 0.0L;
        D(m, k, v) = (((long double)x[k] - z) * prev - m * prevm) / c3;
      }
    }
    for (int m = 0; m <= std::min(k, MD); ++m) {
      const long double prev = D(m, k - 1, k - 1);
      const long double prevm = m > 0 ? D(m - 1, k - 1, k - 1) : 0.0L;
      D(m, k, k) = c1 / c2 * (m * prevm - ((long double)x[k - 1] - z) * prev);
    }
    c1 = c2;
  }
  for (int v = 0; v < n; ++v) {
    w1[v] = (double)D(1, n - 1, v);
    w2[v] = (double)D(2, n - 1, v);
  }
}

template <typename T>
T* dev_alloc(tc_ctx* c, size_t bytes, tc_status& st) {
  void* p = nullptr;
  if (st != TC_OK) return nullptr;
  if (bytes == 0) bytes = 16;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    st = fail(c, TC_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    return nullptr;
  }
  c->bytes += bytes;
  return reinterpret_cast<T*>(p);
}

void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

template <typename T>
void twiddles(int L, std::vector<C2<T>>& out) {
  out.resize(L);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int e = 0; e < L; ++e) {
    const long double ang = -2.0L * pi * (long double)e / (long double)L;
    out[e] = C2<T>{(T)std::cos(ang), (T)std::sin(ang)};
  }
}

void free_ctx(tc_ctx* c) {
  if (!c) return;
  void* ptrs[] = {c->rc_dev, c->fac, c->flin, c->tw_t, c->tw_z, c->twf_t, c->twf_z, c->u, c->u_prev, c->N_prev,
                  c->N_cur, c->p, c->omega, c->aux, c->inter, c->zmax, c->diag_wr, c->diag_uc, c->red};
  for (void* p : ptrs) dev_free(p);
  for (auto& t : c->timers)
    for (auto e : t.ev) (void)hipEventDestroy(e);
  delete c;
}

// One evaluation of the nonlinear term in the convective form: the radial
// derivatives of u, then per plane batch the axial, azimuthal and forward
// axial passes over the 9-field intermediate.
tc_status nonlinear_conv(tc_ctx* c, const cd* u, cd* N) {
  hipError_t e = hipSuccess;
  c->omega_fresh = false;  // the curl buffer holds D1 u here
  timer_begin(c, TK_CURL);
  e = launch_dr(c, u, c->omega);
  timer_end(c, TK_CURL);
  if (e != hipSuccess) return hip_check(c, e, "radial derivatives");
  for (int p0 = 0; p0 < c->d.n_r; p0 += c->batch) {
    const int np = std::min(c->batch, c->d.n_r - p0);
    timer_begin(c, TK_ZINV);
    e = launch_zinv_conv(c, p0, np, u, c->omega);
    timer_end(c, TK_ZINV);
    if (e != hipSuccess) return hip_check(c, e, "axial inverse transform");
    timer_begin(c, TK_THETA);
    e = launch_theta_conv(c, p0, np);
    timer_end(c, TK_THETA);
    if (e != hipSuccess) return hip_check(c, e, "azimuthal transforms");
    timer_begin(c, TK_ZFWD);
    e = launch_zfwd(c, p0, np, N);
    timer_end(c, TK_ZFWD);
    if (e != hipSuccess) return hip_check(c, e, "axial forward transform");
  }
  return TC_OK;
}

// One evaluation of the nonlinear term: u -> N (both 3 fields).
tc_status nonlinear(tc_ctx* c, const cd* u, cd* N) {
  if (c->d.form == TC_CONVECTIVE) return nonlinear_conv(c, u, N);
  hipError_t e = hipSuccess;
  // the previous step's last sweep may already have formed curl(u)
  if (!(u == c->u && c->omega_fresh)) {
    timer_begin(c, TK_CURL);
    e = launch_curl(c, u, c->omega);
    timer_end(c, TK_CURL);
    if (e != hipSuccess) return hip_check(c, e, "curl");
  }
  c->omega_fresh = (u == c->u);
  for (int p0 = 0; p0 < c->d.n_r; p0 += c->batch) {
    const int np = std::min(c->batch, c->d.n_r - p0);
    timer_begin(c, TK_ZINV);
    e = launch_zinv(c, p0, np, u, c->omega);
    timer_end(c, TK_ZINV);
    if (e != hipSuccess) return hip_check(c, e, "axial inverse transform");
    timer_begin(c, TK_THETA);
    e = launch_theta(c, np);
    timer_end(c, TK_THETA);
    if (e != hipSuccess) return hip_check(c, e, "azimuthal transforms");
    timer_begin(c, TK_ZFWD);
    e = launch_zfwd(c, p0, np, N);
    timer_end(c, TK_ZFWD);
    if (e != hipSuccess) return hip_check(c, e, "axial forward transform");
  }
  return TC_OK;
}

size_t field_bytes(const tc_ctx* c) { return (size_t)c->d.F * sizeof(cd); }

}  // namespace

// ---------------------------------------------------------------- diagnostics kernels
namespace tc {

// Per-block partial sums of sum_j w_j r_j sum_{s,n} c_n e(j,s,n), where e is
// the energy density of (u - ref) and ref = circular Couette flow in mode (0,0).
__global__ void k_energy(Dims d, const cd* __restrict__ u, const double* __restrict__ wr, const double* __restrict__ Uc,
                         int subtract, double* __restrict__ partial) {
  __shared__ double red[256];
  double acc = 0.0;
  const int64_t total = d.F;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(idx / d.S);
    const int64_t rem = idx - (int64_t)j * d.S;
    const int s = (int)(rem / d.mt), n = (int)(rem - (int64_t)s * d.mt);
    if (s == d.nyq) continue;
    cd p = u[idx], m = u[d.F + idx], z = u[2 * d.F + idx];
    if (subtract && s == 0 && n == 0) {
      p.y -= Uc[j];
      m.y += Uc[j];
    }
    const double e = 0.5 * (p.x * p.x + p.y * p.y + m.x * m.x + m.y * m.y) + z.x * z.x + z.y * z.y;
    acc += (n == 0 ? 1.0 : 2.0) * wr[j] * e;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Per-block maxima of |div u| over interior nodes (D1 by the 9-point rows).
__global__ void k_divmax(const double* __restrict__ rc, Dims d, const cd* __restrict__ u, double* __restrict__ partial) {
  __shared__ double red[256];
  double mx = 0.0;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < d.S) {
    const int s = (int)(idx / d.mt), n = (int)(idx - (int64_t)s * d.mt);
    if (s != d.nyq) {
      const double a = n * d.kt, b = (s < d.half ? s : s - d.mz) * d.kz;
      for (int i = 1; i < d.n_r - 1; ++i) {
        const double* R = rc + (int64_t)i * RC_N;
        cd dr = {0, 0};
        for (int k = 0; k < NB9; ++k) {
          const int node = i + k - HW;
          if (node < 0 || node >= d.n_r) continue;
          const int64_t o = node * d.S + idx;
          const cd ur = {0.5 * (u[o].x + u[d.F + o].x), 0.5 * (u[o].y + u[d.F + o].y)};
          dr.x += R[RC_W1 + k] * ur.x;
          dr.y += R[RC_W1 + k] * ur.y;
        }
        const int64_t o = i * d.S + idx;
        const cd p = u[o], m = u[d.F + o], z = u[2 * d.F + o];
        const double ir = R[RC_IR];
        const double vx = dr.x + 0.5 * (p.x + m.x) * ir + 0.5 * a * ir * (p.x - m.x) - b * z.y;
        const double vy = dr.y + 0.5 * (p.y + m.y) * ir + 0.5 * a * ir * (p.y - m.y) + b * z.x;
        mx = fmax(mx, sqrt(vx * vx + vy * vy));
      }
    }
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Per-block sums over the inner wall of c_n (|u_theta - Re_i delta|^2 + |u_z|^2).
// Per radial node j (blockIdx.y): block partials of the mode sums
// sum c_n |u_r|, sum c_n |u_theta|, sum c_n |u_z| over the stored modes
// (c_0 = 1, c_n = 2), the bounds of max |u_c| over the (theta, z) plane
// that the CFL estimate of tc_get_diag uses.
__global__ void k_cflsum(Dims d, const cd* __restrict__ u, double* __restrict__ partial) {
  __shared__ double red[3][256];
  const int64_t j = blockIdx.y;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < d.S;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int s = (int)(idx / d.mt), n = (int)(idx - (int64_t)s * d.mt);
    if (s == d.nyq) continue;
    const int64_t o = j * d.S + idx;
    const cd p = u[o], m = u[d.F + o], z = u[2 * d.F + o];
    const double c = n == 0 ? 1.0 : 2.0;
    acc[0] += c * 0.5 * hypot(p.x + m.x, p.y + m.y);  // u_r = (u+ + u-)/2
    acc[1] += c * 0.5 * hypot(p.x - m.x, p.y - m.y);  // |u_theta| = |u+ - u-|/2
    acc[2] += c * hypot(z.x, z.y);
  }
  for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) partial[(j * gridDim.x + blockIdx.x) * 3 + k] = red[k][0];
}

// theta-z mean of u_theta on every node: the real part of the (l, n) = (0, 0)
// coefficient, Re(-i (u+ - u-) / 2) = Im(u+ - u-) / 2.
__global__ void k_mean_utheta(Dims d, const cd* __restrict__ u, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.n_r) return;
  const int64_t o = (int64_t)j * d.S;
  out[j] = 0.5 * (u[o].y - u[d.F + o].y);
}

__global__ void k_slip(Dims d, const cd* __restrict__ u, double* __restrict__ partial) {
  __shared__ double red[256];
  double acc = 0.0;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < d.S) {
    const int s = (int)(idx / d.mt), n = (int)(idx - (int64_t)s * d.mt);
    if (s != d.nyq) {
      const cd p = u[idx], m = u[d.F + idx], z = u[2 * d.F + idx];
      // u_theta = -i (u+ - u-) / 2
      double tx = 0.5 * (p.y - m.y), ty = -0.5 * (p.x - m.x);
      if (s == 0 && n == 0) tx -= d.Re_i;
      acc = (n == 0 ? 1.0 : 2.0) * (tx * tx + ty * ty + z.x * z.x + z.y * z.y);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Gradient of E_pert = 1/2 int |u - U_c|^2 dV (trapezoid rule in r, Parseval
// in theta and z) with respect to the stored coefficients under
// <x, y> = sum Re(conj(x) y):  g+- = (A/2) w_j r_j c_n (u+- - U_c+-),
// g_z = A w_j r_j c_n u_z, A = (2 pi / k_theta)(2 pi / k_z).
__global__ void k_egrad(const double* __restrict__ rc, Dims d, double C1, double C2, double area,
                        const cd* __restrict__ u, cd* __restrict__ g) {
  // (area carries the seed's scale factor)
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.S) return;
  const int s = (int)(idx / d.mt), n = (int)(idx - (int64_t)s * d.mt);
  const int M = d.n_r - 1;
  for (int j = 0; j <= M; ++j) {
    const int64_t o = j * d.S + idx;
    if (s == d.nyq) {
      g[o] = g[d.F + o] = g[2 * d.F + o] = cd{0, 0};
      continue;
    }
    const double r = rc[(int64_t)j * RC_N + RC_R];
    double w = 0.0;
    if (j > 0) w += 0.5 * (r - rc[(int64_t)(j - 1) * RC_N + RC_R]);
    if (j < M) w += 0.5 * (rc[(int64_t)(j + 1) * RC_N + RC_R] - r);
    const double k = area * w * r * (n == 0 ? 1.0 : 2.0);
    cd p = u[o], m = u[d.F + o];
    if (s == 0 && n == 0) {
      const double U = C1 * r + C2 / r;
      p.y -= U;
      m.y += U;
    }
    const cd z = u[2 * d.F + o];
    g[o] = cd{0.5 * k * p.x, 0.5 * k * p.y};
    g[d.F + o] = cd{0.5 * k * m.x, 0.5 * k * m.y};
    g[2 * d.F + o] = cd{k * z.x, k * z.y};
  }
}

__global__ void k_finite(int64_t count, const double* __restrict__ x, int* __restrict__ flag) {
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) bad = 1;
  if (bad) atomicOr(flag, 1);
}

}  // namespace tc


namespace {

// ---------------------------------------------------------------- diagnostics: layout and reduction
// Partial results of the diagnostics kernels, in one array of doubles:
// block partials of the energy, perturbation energy, |div u| maximum and
// slip sums, the CFL mode sums per radial node, and the theta-z mean of
// u_theta on every node.
struct DiagLayout {
  int nb, nbd, np, nbc;
  size_t ncfl, o00, total;
};

DiagLayout diag_layout(const Dims& d) {
  DiagLayout L;
  L.nb = 1024;
  L.nbd = (int)((d.S + 255) / 256);
  L.np = std::max(L.nb, L.nbd);
  L.nbc = 32;  // blocks per radial node of the CFL sums
  L.ncfl = (size_t)d.n_r * L.nbc * 3;
  L.o00 = 4 * (size_t)L.np + L.ncfl;
  L.total = L.o00 + (size_t)d.n_r;
  return L;
}

hipError_t diag_launch(tc_ctx* c, double* part, const DiagLayout& L) {
  const Dims& d = c->d;
  hipLaunchKernelGGL(k_energy, dim3(L.nb), dim3(256), 0, c->stream, d, c->u, c->diag_wr, c->diag_uc, 0, part);
  hipLaunchKernelGGL(k_energy, dim3(L.nb), dim3(256), 0, c->stream, d, c->u, c->diag_wr, c->diag_uc, 1, part + L.np);
  hipLaunchKernelGGL(k_divmax, dim3(L.nbd), dim3(256), 0, c->stream, c->rc_dev, d, c->u, part + 2 * L.np);
  hipLaunchKernelGGL(k_slip, dim3(L.nbd), dim3(256), 0, c->stream, d, c->u, part + 3 * L.np);
  hipLaunchKernelGGL(k_cflsum, dim3(L.nbc, d.n_r), dim3(256), 0, c->stream, d, c->u, part + 4 * L.np);
  hipLaunchKernelGGL(k_mean_utheta, dim3((d.n_r + 255) / 256), dim3(256), 0, c->stream, d, c->u, part + L.o00);
  return hipGetLastError();
}

// The eight diagnostics from the partials h (layout L) and the per-node
// constants rc.  One source for the host reduction of tc_get_diag and the
// device one of tc_get_diag_noalloc: with contraction off, both evaluate
// the same operations in the same order and agree bit for bit.
__host__ __device__ void diag_reduce(const Dims& d, const DiagLayout& L, const double* h, const double* rc, double eta,
                                     double* out) {
#pragma clang fp contract(off)
  const double pi = 3.14159265358979323846;
  const double area = (2.0 * pi / d.kt) * (2.0 * pi / d.kz);
  double E = 0, Ep = 0, dv = 0, sl = 0;
  for (int i = 0; i < L.nb; ++i) {
    E += h[i];
    Ep += h[L.np + i];
  }
  for (int i = 0; i < L.nbd; ++i) {
    dv = dv > h[2 * L.np + i] ? dv : h[2 * L.np + i];
    sl += h[3 * L.np + i];
  }
  out[0] = 0.5 * area * E;
  out[1] = 0.5 * area * Ep;
  out[2] = dv;
  out[3] = sqrt(sl) / fabs(d.Re_i == 0.0 ? 1.0 : d.Re_i);
  // CFL bound: dt max_j (B_r/dr_j + B_theta/(r_j dtheta) + B_z/dz) on the
  // physical grid (2 m_theta, m_z), dr_j the distance to the nearer neighbour
  const double dth = 2.0 * pi / (d.kt * 2.0 * d.mt), dz = 2.0 * pi / (d.kz * d.mz);
  auto R = [&](int j) { return rc[(size_t)j * RC_N + RC_R]; };
  double cfl = 0.0;
  for (int j = 0; j < d.n_r; ++j) {
    double B[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < L.nbc; ++b)
      for (int k = 0; k < 3; ++k) B[k] += h[4 * (size_t)L.np + ((size_t)j * L.nbc + b) * 3 + k];
    double dr = HUGE_VAL;
    if (j > 0) dr = fmin(dr, R(j) - R(j - 1));
    if (j + 1 < d.n_r) dr = fmin(dr, R(j + 1) - R(j));
    const double v = B[0] / dr + B[1] / (R(j) * dth) + B[2] / dz;
    cfl = cfl > v ? cfl : v;
  }
  out[4] = d.dt * cfl;
  out[5] = 0.0;  // the step count is filled in by the caller
  // Quasi-Nusselt numbers: r^3 d<omega>/dr at each wall over its Couette
  // value -2 C2, <omega> = <u_theta>/r, d/dr by the wall rows of D1
  const int M = d.n_r - 1;
  const double C2 = eta * (d.Re_i - eta * d.Re_o) / ((1.0 - eta) * (1.0 - eta * eta));
  if (C2 == 0.0) {
    out[6] = out[7] = NAN;
  } else {
    for (int w = 0; w < 2; ++w) {
      const int j = w ? M : 0;
      const int lo = j - HW < 0 ? 0 : j - HW, hi = j + HW > M ? M : j + HW;
      double dw = 0.0;
      for (int k = lo; k <= hi; ++k) dw += rc[(size_t)j * RC_N + RC_W1 + (k - j + HW)] * (h[L.o00 + k] / R(k));
      out[6 + w] = R(j) * R(j) * R(j) * dw / (-2.0 * C2);
    }
  }
}

__global__ void k_diag_finish(Dims d, DiagLayout L, const double* part, const double* rc, double eta, double* out) {
  diag_reduce(d, L, part, rc, eta, out);
}

// Scratch of tc_get_diag_noalloc: one array per GPU, from module load to
// process end.  Host code takes its device address per device from
// hipGetSymbolAddress (tc_init, with the context's device current) and
// never uses the array's name.
static __device__ __align__(256) double scratch[TC_DIAG_SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
double* g_scratch[MAX_DEVICES] = {};

// Device address of the scratch on the current device (looked up once per
// device); nullptr if the lookup fails.
double* scratch_address(int dev) {
  static std::mutex m;
  std::lock_guard<std::mutex> lk(m);
  if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch[dev] = static_cast<double*>(ptr);
  }
  return g_scratch[dev];
}

double* diag_scratch(const tc_ctx* c) {
  return (c->device >= 0 && c->device < MAX_DEVICES) ? g_scratch[c->device] : nullptr;
}

}  // namespace

namespace tc {

hipError_t energy_of(tc_ctx* c, const cd* u, double& E) {
  const int nb = 1024;
  hipLaunchKernelGGL(k_energy, dim3(nb), dim3(256), 0, c->stream, c->d, u, c->diag_wr, c->diag_uc, 0, c->red);
  hipError_t e = hipGetLastError();
  std::vector<double> h(nb, 0.0);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), c->red, nb * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  double sum = 0.0;
  for (int i = 0; i < nb; ++i) sum += h[i];
  const double area = (2.0 * M_PI / c->d.kt) * (2.0 * M_PI / c->d.kz);
  E = 0.5 * area * sum;
  return e;
}

}  // namespace tc

// ================================================================== C ABI
extern "C" {

const char* tc_last_error(const tc_ctx* ctx) {
  if (!ctx) return g_init_error.c_str();
  return ctx->err.c_str();
}

// smallest supported transform length >= L (0 if there is none)
static int fft_length_at_least(int L) {
  for (int x = L < 1 ? 1 : L; x <= 2048; ++x)
    if (fft_length_supported(x)) return x;
  return 0;
}

tc_status tc_init(const tc_grid* g, double eta, double Re_i, double Re_o, double dt, void* hip_stream,
                  tc_ctx** out) {
  g_init_error.clear();
  if (!out) {
    g_init_error = "out is NULL";
    return TC_EINVAL;
  }
  *out = nullptr;
  if (!g) {
    g_init_error = "grid is NULL";
    return TC_EINVAL;
  }
  tc_grid G = *g;
  // default dealiased grid: the smallest supported length that meets the
  // 3/2 rule (0 when the rule asks for more than the longest one, which the
  // length check below then rejects)
  if (G.p_theta == 0) G.p_theta = fft_length_at_least(3 * G.m_theta - 2);
  if (G.p_z == 0) G.p_z = fft_length_at_least(3 * G.m_z / 2 - 2);
  std::string why;
  if (G.n_r < 9 || G.n_r > 4096) why = "n_r must be in [9, 4096]";
  else if (G.m_theta < 1 || G.m_z < 2 || (G.m_z % 2)) why = "m_theta >= 1 and even m_z >= 2 required";
  else if (G.n_s != 9) why = "only n_s = 9 is supported";
  else if (G.precision != TC_FP64 && G.precision != TC_FP32_BULK) why = "unknown precision";
  else if (G.form != TC_ROTATIONAL && G.form != TC_CONVECTIVE) why = "unknown form of the nonlinear term";
  else if (G.form == TC_CONVECTIVE && G.precision != TC_FP64) why = "the convective form runs in FP64 only";
  else if (G.p_theta < 3 * G.m_theta - 2 || G.p_z < 3 * G.m_z / 2 - 2) why = "dealiased grid below the 3/2 rule";
  else if (!fft_length_supported(G.p_theta) || !fft_length_supported(G.p_z)) why = "unsupported transform length";
  else if (!(eta > 0.0 && eta < 1.0)) why = "eta must be in (0, 1)";
  else if (!(dt > 0.0) || !std::isfinite(dt)) why = "dt must be positive";
  else if (!(G.k_theta > 0.0) || !(G.k_z > 0.0)) why = "k_theta, k_z must be positive";
  else if (!(G.alpha >= 0.0 && G.alpha <= 1.0)) why = "alpha must be in [0, 1]";
  else if (!std::isfinite(Re_i) || !std::isfinite(Re_o)) why = "Reynolds numbers must be finite";
  if (!why.empty()) {
    g_init_error = why;
    return TC_EINVAL;
  }

  tc_ctx* c = new (std::nothrow) tc_ctx();
  if (!c) {
    g_init_error = "out of host memory";
    return TC_ENOMEM;
  }
  c->g = G;
  c->eta = eta;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->r_i = eta / (1.0 - eta);
  c->r_o = 1.0 / (1.0 - eta);
  Dims& d = c->d;
  d.n_r = G.n_r;
  d.mt = G.m_theta;
  d.mz = G.m_z;
  d.pt = G.p_theta;
  d.pz = G.p_z;
  d.half = G.m_z / 2;
  d.nyq = G.m_z / 2;
  d.ndm = G.m_theta * (G.m_z / 2);
  d.S = (int64_t)G.m_z * G.m_theta;
  d.F = (int64_t)G.n_r * d.S;
  d.kt = G.k_theta;
  d.kz = G.k_z;
  d.dt = dt;
  d.Re_i = Re_i;
  d.Re_o = Re_o;
  d.form = G.form;

  // radial grid and per-node constants
  c->r = radial_nodes(d.n_r, eta, G.alpha);
  const int M = d.n_r - 1;
  c->rc.assign((size_t)d.n_r * RC_N, 0.0);
  for (int j = 0; j < d.n_r; ++j) {
    double* R = &c->rc[(size_t)j * RC_N];
    R[RC_R] = c->r[j];
    R[RC_IR] = 1.0 / c->r[j];
    R[RC_IR2] = 1.0 / (c->r[j] * c->r[j]);
    const int lo = std::max(0, j - HW), hi = std::min(M, j + HW);
    double w1[NB9], w2[NB9];
    fd_weights(c->r[j], &c->r[lo], hi - lo + 1, w1, w2);
    for (int k = lo; k <= hi; ++k) {
      R[RC_W1 + (k - j + HW)] = w1[k - lo];
      R[RC_W2 + (k - j + HW)] = w2[k - lo];
    }
  }
  // Neumann rows of P scaled to the size of the adjacent Laplacian rows
  auto rowmax = [&](int j, int off) {
    double m = 0.0;
    for (int k = 0; k < NB9; ++k) m = std::max(m, std::fabs(c->rc[(size_t)j * RC_N + off + k]));
    return m;
  };
  d.s0 = rowmax(1, RC_W2) / rowmax(0, RC_W1);
  d.sM = rowmax(M - 1, RC_W2) / rowmax(M, RC_W1);

  tc_status st = TC_OK;
  const size_t FB = field_bytes(c);
  c->rc_dev = dev_alloc<double>(c, c->rc.size() * sizeof(double), st);
  c->fac = dev_alloc<double>(c, (size_t)NOPS * d.n_r * NFAC * d.ndm * sizeof(double), st);
  // the line predictor-corrector where the grid allows it (TC_PC_LINE=0
  // selects the four-sweep kernels instead)
  {
    const char* e = std::getenv("TC_PC_LINE");
    if (line_lps(d) > 0 && !(e && std::atoi(e) == 0))
      c->flin = dev_alloc<double>(c, (size_t)NOPS * d.n_r * NFAC * d.ndm * sizeof(double), st);
  }
  // the curl adjoint as one radial sweep per slot where there are enough
  // slots for the GPU (at least 2048 waves); TC_ADJ_CURL_SWEEP=0 or 1 at
  // this call chooses the tiled or the sweep form on any grid
  {
    const char* e = std::getenv("TC_ADJ_CURL_SWEEP");
    c->adj_curl_sweep = e ? std::atoi(e) != 0 : d.S >= 131072;
  }
  c->tw_t = dev_alloc<cd>(c, (size_t)d.pt * sizeof(cd), st);
  c->tw_z = dev_alloc<cd>(c, (size_t)d.pz * sizeof(cd), st);
  c->twf_t = dev_alloc<cf>(c, (size_t)d.pt * sizeof(cf), st);
  c->twf_z = dev_alloc<cf>(c, (size_t)d.pz * sizeof(cf), st);
  c->u = dev_alloc<cd>(c, 3 * FB, st);
  c->u_prev = dev_alloc<cd>(c, 3 * FB, st);
  c->N_prev = dev_alloc<cd>(c, 3 * FB, st);
  c->N_cur = dev_alloc<cd>(c, 3 * FB, st);
  c->p = dev_alloc<cd>(c, FB, st);
  c->omega = dev_alloc<cd>(c, 3 * FB, st);
  c->zmax = dev_alloc<unsigned int>(c, (size_t)ZMAX_WORDS * d.n_r * sizeof(unsigned int), st);
  c->diag_wr = dev_alloc<double>(c, (size_t)d.n_r * sizeof(double), st);
  c->diag_uc = dev_alloc<double>(c, (size_t)d.n_r * sizeof(double), st);
  c->red = dev_alloc<double>(c, TC_RED_DOUBLES * sizeof(double), st);
  // plane batch of the nonlinear term: all planes when they fit a budget
  {
    const size_t per = inter_bytes_per_plane(c);
    size_t budget = (size_t)48 << 30;
    if (const char* e = std::getenv("TC_BATCH_PLANES")) c->batch = std::max(1, std::atoi(e));
    else c->batch = (int)std::max<size_t>(1, std::min<size_t>((size_t)d.n_r, budget / std::max<size_t>(per, 1)));
    c->batch = std::min(c->batch, d.n_r);
    c->inter = dev_alloc<void>(c, per * (size_t)c->batch, st);
  }
  if (st != TC_OK) {
    g_init_error = c->err;
    free_ctx(c);
    return st;
  }
  std::vector<cd> tw;
  std::vector<cf> twf;
  hipError_t e = hipSuccess;
  auto up = [&](void* dst, const void* src, size_t n) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, c->stream);
  };
  up(c->rc_dev, c->rc.data(), c->rc.size() * sizeof(double));
  // energy weights w_j r_j (trapezoid rule) and the Couette profile, for
  // the diagnostics
  std::vector<double> wr(d.n_r, 0.0), Uc(d.n_r);
  {
    for (int j = 0; j + 1 < d.n_r; ++j) {
      const double h = c->r[j + 1] - c->r[j];
      wr[j] += 0.5 * h;
      wr[j + 1] += 0.5 * h;
    }
    const double C1 = (d.Re_o - eta * d.Re_i) / (1.0 + eta);
    const double C2 = eta * (d.Re_i - eta * d.Re_o) / ((1.0 - eta) * (1.0 - eta * eta));
    for (int j = 0; j < d.n_r; ++j) {
      wr[j] *= c->r[j];
      Uc[j] = C1 * c->r[j] + C2 / c->r[j];
    }
  }
  up(c->diag_wr, wr.data(), wr.size() * sizeof(double));
  up(c->diag_uc, Uc.data(), Uc.size() * sizeof(double));
  // twiddle tables (separate host vectors: the copies are asynchronous)
  std::vector<cd> tw_t, tw_z;
  std::vector<cf> twf_t, twf_z;
  twiddles<double>(d.pt, tw_t);
  twiddles<double>(d.pz, tw_z);
  twiddles<float>(d.pt, twf_t);
  twiddles<float>(d.pz, twf_z);
  up(c->tw_t, tw_t.data(), tw_t.size() * sizeof(cd));
  up(c->tw_z, tw_z.data(), tw_z.size() * sizeof(cd));
  up(c->twf_t, twf_t.data(), twf_t.size() * sizeof(cf));
  up(c->twf_z, twf_z.data(), twf_z.size() * sizeof(cf));
  if (e == hipSuccess) e = hipMemsetAsync(c->u, 0, 3 * FB, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->u_prev, 0, 3 * FB, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->N_prev, 0, 3 * FB, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->N_cur, 0, 3 * FB, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->p, 0, FB, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->zmax, 0, (size_t)ZMAX_WORDS * d.n_r * sizeof(unsigned int), c->stream);
  int* bad = nullptr;
  if (e == hipSuccess) e = hipMalloc(&bad, sizeof(int));
  if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int), c->stream);
  if (e == hipSuccess) e = launch_factor(c, bad);
  int hbad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (bad) (void)hipFree(bad);
  if (e != hipSuccess) {
    g_init_error = std::string("HIP error during set-up: ") + hipGetErrorString(e);
    free_ctx(c);
    return TC_EHIP;
  }
  if (hbad) {
    g_init_error = "zero or non-finite pivot in the banded factorisation";
    free_ctx(c);
    return TC_ESINGULAR;
  }
  // the factors are unpivoted: check their backward error on one solve per
  // operator and mode before accepting them
  {
    double* tmp = nullptr;
    unsigned long long* worst = nullptr;
    unsigned long long hw = 0;
    const size_t tb = (size_t)d.n_r * NOPS * d.ndm * sizeof(double);
    if (hipMalloc(&tmp, tb) != hipSuccess || hipMalloc(&worst, sizeof(*worst)) != hipSuccess) {
      (void)hipGetLastError();
      if (tmp) (void)hipFree(tmp);
      g_init_error = "hipMalloc of the factor check's work space failed";
      free_ctx(c);
      return TC_ENOMEM;
    }
    e = hipMemsetAsync(worst, 0, sizeof(*worst), c->stream);
    if (e == hipSuccess) e = launch_factor_check(c, tmp, worst);
    if (e == hipSuccess) e = hipMemcpyAsync(&hw, worst, sizeof(hw), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(tmp);
    (void)hipFree(worst);
    if (e != hipSuccess) {
      g_init_error = std::string("HIP error during the factor check: ") + hipGetErrorString(e);
      free_ctx(c);
      return TC_EHIP;
    }
    std::memcpy(&c->factor_error, &hw, sizeof(double));
    if (!(c->factor_error <= TC_FACTOR_CHECK_MAX)) {
      g_init_error = "the unpivoted factors fail the backward-error check (" + std::to_string(c->factor_error) + ")";
      free_ctx(c);
      return TC_ESINGULAR;
    }
  }
  // the allocation-free diagnostics' scratch address on this device
  if (hipGetDevice(&c->device) != hipSuccess || !scratch_address(c->device)) {
    (void)hipGetLastError();
    g_init_error = "cannot look up the diagnostics scratch on this device";
    free_ctx(c);
    return TC_EHIP;
  }
  *out = c;
  return TC_OK;
}

tc_status tc_destroy(tc_ctx* ctx) {
  if (!ctx) return TC_EINVAL;
  (void)hipStreamSynchronize(ctx->stream);
  free_ctx(ctx);
  return TC_OK;
}

tc_status tc_radial_nodes(const tc_ctx* ctx, double* r_host) {
  if (!ctx || !r_host) return TC_EINVAL;
  std::memcpy(r_host, ctx->r.data(), ctx->r.size() * sizeof(double));
  return TC_OK;
}

tc_status tc_set_state(tc_ctx* c, const void* u, const void* u_prev, const void* N_prev) {
  if (!c) return TC_EINVAL;
  if (!u) return fail(c, TC_EINVAL, "u is NULL");
  const size_t B3 = 3 * field_bytes(c);
  c->omega_fresh = false;
  hipError_t e = hipMemcpyAsync(c->u, u, B3, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->u_prev, u_prev ? u_prev : u, B3, hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_check(c, e, "tc_set_state copy");
  if (N_prev) {
    e = hipMemcpyAsync(c->N_prev, N_prev, B3, hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_check(c, e, "tc_set_state copy");
  } else {
    tc_status s = nonlinear(c, c->u_prev, c->N_prev);
    if (s != TC_OK) return s;
  }
  e = hipMemsetAsync(c->p, 0, field_bytes(c), c->stream);
  if (e != hipSuccess) return hip_check(c, e, "tc_set_state");
  c->steps = 0;
  c->have_p = false;
  return TC_OK;
}

tc_status tc_get_state(const tc_ctx* cc, void* u, void* p) {
  tc_ctx* c = const_cast<tc_ctx*>(cc);
  if (!c) return TC_EINVAL;
  if (!u && !p) return fail(c, TC_EINVAL, "nothing to copy");
  hipError_t e = hipSuccess;
  if (u) e = hipMemcpyAsync(u, c->u, 3 * field_bytes(c), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && p) e = hipMemcpyAsync(p, c->p, field_bytes(c), hipMemcpyDeviceToDevice, c->stream);
  return hip_check(c, e, "tc_get_state copy");
}

tc_status tc_get_history(const tc_ctx* cc, void* u_prev, void* N_prev) {
  tc_ctx* c = const_cast<tc_ctx*>(cc);
  if (!c) return TC_EINVAL;
  hipError_t e = hipSuccess;
  if (u_prev) e = hipMemcpyAsync(u_prev, c->u_prev, 3 * field_bytes(c), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && N_prev)
    e = hipMemcpyAsync(N_prev, c->N_prev, 3 * field_bytes(c), hipMemcpyDeviceToDevice, c->stream);
  return hip_check(c, e, "tc_get_history copy");
}

tc_status tc_step(tc_ctx* c, int32_t nsteps) {
  if (!c) return TC_EINVAL;
  if (nsteps < 0) return fail(c, TC_EINVAL, "nsteps must be >= 0");
  if (c->timing)
    for (auto& t : c->timers) t.used = 0;
  for (int32_t k = 0; k < nsteps; ++k) {
    tc_status s = nonlinear(c, c->u, c->N_cur);
    if (s != TC_OK) return s;
    timer_begin(c, TK_PC);
    hipError_t e = launch_pc(c, c->u, c->u_prev, c->N_cur, c->N_prev, c->u_prev, c->p, k == nsteps - 1, c->omega);
    timer_end(c, TK_PC);
    if (e != hipSuccess) return hip_check(c, e, "predictor-corrector");
    std::swap(c->u, c->u_prev);
    std::swap(c->N_cur, c->N_prev);
    c->omega_fresh = pc_fuses_curl(c);  // then omega = curl(u^{i+1})
    ++c->steps;
    c->have_p = true;
  }
  return TC_OK;
}

tc_status tc_nonlinear(tc_ctx* c, const void* u, void* N) {
  if (!c) return TC_EINVAL;
  if (!u || !N) return fail(c, TC_EINVAL, "NULL array");
  const char* a = static_cast<const char*>(u);
  const char* b = static_cast<const char*>(N);
  const size_t B3 = 3 * field_bytes(c);
  if (a < b + B3 && b < a + B3) return fail(c, TC_EINVAL, "u and N overlap");
  return nonlinear(c, static_cast<const cd*>(u), static_cast<cd*>(N));
}

static int op_of(tc_solve_kind k) {
  switch (k) {
    case TC_SOLVE_P:
    case TC_SOLVE_PHI: return OP_P;
    case TC_SOLVE_UPLUS: return OP_HP;
    case TC_SOLVE_UMINUS: return OP_HM;
    case TC_SOLVE_UZ: return OP_HZ;
  }
  return -1;
}

tc_status tc_helmholtz_solve(tc_ctx* c, tc_solve_kind k, const void* rhs, void* x) {
  if (!c) return TC_EINVAL;
  const int op = op_of(k);
  if (op < 0) return fail(c, TC_EINVAL, "unknown solve kind");
  if (!rhs || !x) return fail(c, TC_EINVAL, "NULL array");
  return hip_check(c, launch_solve(c, op, 0, static_cast<const cd*>(rhs), static_cast<cd*>(x)), "solve");
}

tc_status tc_helmholtz_solve_transposed(tc_ctx* c, tc_solve_kind k, const void* rhs, void* x) {
  if (!c) return TC_EINVAL;
  const int op = op_of(k);
  if (op < 0) return fail(c, TC_EINVAL, "unknown solve kind");
  if (!rhs || !x) return fail(c, TC_EINVAL, "NULL array");
  if (rhs == x) return fail(c, TC_EINVAL, "the transposed solve needs x != rhs");
  return hip_check(c, launch_solve(c, op, 1, static_cast<const cd*>(rhs), static_cast<cd*>(x)), "solve");
}

tc_status tc_get_diag(tc_ctx* c, double* out) {
  if (!c || !out) return TC_EINVAL;
  const DiagLayout L = diag_layout(c->d);
  double* part = nullptr;
  hipError_t e = hipMalloc(&part, L.total * sizeof(double));
  if (e == hipSuccess) e = diag_launch(c, part, L);
  std::vector<double> h(L.total, 0.0);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), part, L.total * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(part);
  if (e != hipSuccess) return hip_check(c, e, "tc_get_diag");
  diag_reduce(c->d, L, h.data(), c->rc.data(), c->eta, out);
  out[5] = (double)c->steps;
  return TC_OK;
}

tc_status tc_get_diag_noalloc(tc_ctx* c, double* out) {
  if (!c || !out) return TC_EINVAL;
  const DiagLayout L = diag_layout(c->d);
  if (L.total + 8 > TC_DIAG_SCRATCH_DOUBLES)
    return fail(c, TC_EINVAL, "tc_get_diag_noalloc: the grid needs " + std::to_string(L.total + 8) +
                                  " doubles of scratch, more than its " + std::to_string(TC_DIAG_SCRATCH_DOUBLES));
  double* part = diag_scratch(c);
  if (!part) return fail(c, TC_EHIP, "tc_get_diag_noalloc: no scratch address for this device");
  hipError_t e = diag_launch(c, part, L);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(1), 0, c->stream, c->d, L, part, c->rc_dev, c->eta,
                       part + L.total);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, part + L.total, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_check(c, e, "tc_get_diag_noalloc");
  out[5] = (double)c->steps;
  return TC_OK;
}

tc_status tc_adjoint_seed(tc_ctx* c, const void* u, double scale, void* g) {
  if (!c) return TC_EINVAL;
  if (!u || !g) return fail(c, TC_EINVAL, "NULL array");
  if (!std::isfinite(scale)) return fail(c, TC_EINVAL, "scale must be finite");
  const Dims& d = c->d;
  const double C1 = (d.Re_o - c->eta * d.Re_i) / (1.0 + c->eta);
  const double C2 = c->eta * (d.Re_i - c->eta * d.Re_o) / ((1.0 - c->eta) * (1.0 - c->eta * c->eta));
  const double area = scale * (2.0 * M_PI / d.kt) * (2.0 * M_PI / d.kz);
  hipLaunchKernelGGL(k_egrad, dim3((unsigned)((d.S + 255) / 256)), dim3(256), 0, c->stream, c->rc_dev, d, C1, C2,
                     area, static_cast<const cd*>(u), static_cast<cd*>(g));
  return hip_check(c, hipGetLastError(), "tc_adjoint_seed");
}

tc_status tc_perturbation_energy_gradient(tc_ctx* c, const void* u, void* g) {
  if (!c) return TC_EINVAL;
  if (!u || !g) return fail(c, TC_EINVAL, "NULL array");
  const Dims& d = c->d;
  const double C1 = (d.Re_o - c->eta * d.Re_i) / (1.0 + c->eta);
  const double C2 = c->eta * (d.Re_i - c->eta * d.Re_o) / ((1.0 - c->eta) * (1.0 - c->eta * c->eta));
  const double area = (2.0 * M_PI / d.kt) * (2.0 * M_PI / d.kz);
  hipLaunchKernelGGL(k_egrad, dim3((unsigned)((d.S + 255) / 256)), dim3(256), 0, c->stream, c->rc_dev, d, C1, C2,
                     area, static_cast<const cd*>(u), static_cast<cd*>(g));
  return hip_check(c, hipGetLastError(), "tc_perturbation_energy_gradient");
}

tc_status tc_check_finite(tc_ctx* c) {
  if (!c) return TC_EINVAL;
  int* flag = nullptr;
  int h = 0;
  hipError_t e = hipMalloc(&flag, sizeof(int));
  if (e == hipSuccess) e = hipMemsetAsync(flag, 0, sizeof(int), c->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_finite, dim3(2048), dim3(256), 0, c->stream, (int64_t)6 * c->d.F,
                       reinterpret_cast<const double*>(c->u), flag);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (flag) (void)hipFree(flag);
  if (e != hipSuccess) return hip_check(c, e, "tc_check_finite");
  return h ? fail(c, TC_ENONFINITE, "non-finite value in the velocity") : TC_OK;
}

tc_status tc_set_timing(tc_ctx* c, int32_t enable) {
  if (!c) return TC_EINVAL;
  c->timing = enable != 0;
  for (auto& t : c->timers) t.used = 0;
  return TC_OK;
}

tc_status tc_kernel_time(tc_ctx* c, int32_t which, double* ms_out, int32_t* launches_out) {
  if (!c || !ms_out || which < 0 || which >= TK_N) return TC_EINVAL;
  KernelTimer& t = c->timers[which];
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_check(c, e, "tc_kernel_time");
  double tot = 0.0;
  int n = 0;
  for (int i = 0; i + 1 < t.used; i += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.ev[i], t.ev[i + 1]) == hipSuccess) {
      tot += ms;
      ++n;
    }
  }
  *ms_out = n ? tot / n : 0.0;
  if (launches_out) *launches_out = n;
  return TC_OK;
}

tc_status tc_factor_backward_error(const tc_ctx* c, double* out) {
  if (!c || !out) return TC_EINVAL;
  *out = c->factor_error;
  return TC_OK;
}

tc_status tc_memory_bytes(const tc_ctx* c, uint64_t* out) {
  if (!c || !out) return TC_EINVAL;
  *out = c->bytes;
  return TC_OK;
}

}  // extern "C"
