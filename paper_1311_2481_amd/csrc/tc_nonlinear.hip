// Pseudospectral nonlinear term N = omega x u with 3/2 dealiasing (Sec. 3.2,
// step 1 of the paper, rotational form).
//
// Complex-pair formulation.  With h = v_r + i v_theta, the full (+-n)
// spectrum of h is  v+ (n >= 0)  and  conj(v-(-l, -n))  (n < 0), so u_r,
// u_theta come out of ONE complex transform of (u+, u-), and likewise
// omega_r, omega_theta from (omega+, omega-); u_z and omega_z are packed as
// g = u_z + i omega_z.  In physical space
//     N_r + i N_theta = i (omega_z h_u - u_z h_omega),
//     N_z             = Im(conj(h_omega) h_u),
// and the forward transform of N_r + i N_theta yields N+ on n >= 0 and
// conj(N-(-l,-n)) on n < 0.  No +-/(r,theta) conversion is ever needed.
// At n = 0 the two stored copies of a real field's coefficients (u+(l) and
// conj(u-(-l))) are averaged, and the imaginary parts of u_z, omega_z are
// dropped, which is what a real-to-complex transform does with an n = 0
// bin: the result equals the plain transform of the cylindrical components
// for every input, Hermitian or not.
//
// Kernels, per batch of radial planes:
//   k_curl  : omega+, omega-, omega_z from u (radial D1 by the 9-point stencil),
//             one lane per (l, n) marching through the radial nodes.
//   k_zinv  : zero-pad and inverse-transform along z the 6 spectral fields
//             (u+, u-, u_z, omega+, omega-, omega_z), NF columns per workgroup.
//   k_theta : per z-row: assemble the 3 complex theta spectra, inverse
//             transforms, products, forward transforms; writes the
//             z-partial spectra of N+, N-, N_z over the first three inputs.
//   k_zfwd  : forward z-transform, 1/(P_theta P_z) scaling, truncation to
//             the stored modes.
// Transform precision T is double, or float in the FP32-bulk form (the
// spectral inputs and outputs stay double).
#include "tc_internal.h"

namespace tc {

// ------------------------------------------------------------------ curl
// KIND 0: omega = curl u; KIND 1: the radial derivatives D1 u+, D1 u-, D1 u_z
// that the convective form transforms.
template <int KIND>
__global__ __launch_bounds__(256) void k_curl(const double* __restrict__ rc, Dims d, const cd* __restrict__ u,
                                              cd* __restrict__ w) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d.S) return;
  const int s = (int)(idx / d.mt), n = (int)(idx - (int64_t)s * d.mt);
  const int M = d.n_r - 1;
  const int64_t F = d.F, S = d.S;
  if (s == d.nyq) {
    for (int j = 0; j <= M; ++j) {
      w[j * S + idx] = cd{0, 0};
      w[F + j * S + idx] = cd{0, 0};
      w[2 * F + j * S + idx] = cd{0, 0};
    }
    return;
  }
  const double a = n * d.kt;
  const double b = (s < d.half ? s : s - d.mz) * d.kz;
  cd wp[NB9], wm[NB9], wz[NB9];
  for (int k = 0; k < NB9; ++k) wp[k] = wm[k] = wz[k] = cd{0, 0};
  for (int j = 0; j <= M + HW; ++j) {
    for (int k = 0; k < NB9 - 1; ++k) { wp[k] = wp[k + 1]; wm[k] = wm[k + 1]; wz[k] = wz[k + 1]; }
    if (j <= M) {
      const int64_t o = j * S + idx;
      wp[NB9 - 1] = u[o]; wm[NB9 - 1] = u[F + o]; wz[NB9 - 1] = u[2 * F + o];
    } else {
      wp[NB9 - 1] = wm[NB9 - 1] = wz[NB9 - 1] = cd{0, 0};
    }
    const int i = j - HW;
    if (i < 0) continue;
    const double* R = rc + (int64_t)i * RC_N;
    const double ir = R[RC_IR];
    cd dp = {0, 0}, dmn = {0, 0}, dz = {0, 0};
#pragma unroll
    for (int k = 0; k < NB9; ++k) {
      const double c = R[RC_W1 + k];
      dp.x = fma(c, wp[k].x, dp.x); dp.y = fma(c, wp[k].y, dp.y);
      dmn.x = fma(c, wm[k].x, dmn.x); dmn.y = fma(c, wm[k].y, dmn.y);
      dz.x = fma(c, wz[k].x, dz.x); dz.y = fma(c, wz[k].y, dz.y);
    }
    const int64_t o = i * S + idx;
    if constexpr (KIND == 1) {
      w[o] = dp;
      w[F + o] = dmn;
      w[2 * F + o] = dz;
      continue;
    }
    const cd up = wp[HW], um = wm[HW], uz = wz[HW];
    // omega+ = i (a/r uz - D1 uz) - b u+ ;  omega- = i (a/r uz + D1 uz) + b u-
    const cd tp = {a * ir * uz.x - dz.x, a * ir * uz.y - dz.y};
    const cd tm = {a * ir * uz.x + dz.x, a * ir * uz.y + dz.y};
    const cd op = {-tp.y - b * up.x, tp.x - b * up.y};
    const cd om = {-tm.y + b * um.x, tm.x + b * um.y};
    // omega_z = -(i/2) [ (D1 + (1+a)/r) u+ - (D1 + (1-a)/r) u- ]
    const cd q = {dp.x + (1.0 + a) * ir * up.x - dmn.x - (1.0 - a) * ir * um.x,
                  dp.y + (1.0 + a) * ir * up.y - dmn.y - (1.0 - a) * ir * um.y};
    const cd oz = {0.5 * q.y, -0.5 * q.x};
    w[o] = op;
    w[F + o] = om;
    w[2 * F + o] = oz;
  }
}

// The same curl with one thread per (radial node, slot) point (grid: x over
// slots, y over nodes): each thread applies row k of D1 to the 9 rows
// around it.  For small grids, where the marching kernel has too few lanes
// to hide memory latency; the rows it re-reads are then cache resident.
template <int KIND>
__global__ __launch_bounds__(256) void k_curl_points(const double* __restrict__ rc, Dims d, const cd* __restrict__ u,
                                                     cd* __restrict__ w) {
  const unsigned idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (unsigned)d.S) return;
  const int k = blockIdx.y;
  const int M = d.n_r - 1;
  const int64_t F = d.F, S = d.S;
  const int64_t o = k * S + idx;
  const int s = (int)(idx / (unsigned)d.mt), n = (int)(idx - (unsigned)s * (unsigned)d.mt);
  if (s == d.nyq) {
    w[o] = cd{0, 0};
    w[F + o] = cd{0, 0};
    w[2 * F + o] = cd{0, 0};
    return;
  }
  const double a = n * d.kt;
  const double b = (s < d.half ? s : s - d.mz) * d.kz;
  const double* R = rc + (int64_t)k * RC_N;
  const double ir = R[RC_IR];
  cd dp = {0, 0}, dmn = {0, 0}, dz = {0, 0};
#pragma unroll
  for (int t = 0; t < NB9; ++t) {
    const int i = k - HW + t;
    if (i < 0 || i > M) continue;
    const double c = R[RC_W1 + t];
    const int64_t oi = i * S + idx;
    const cd p = u[oi], m = u[F + oi], z = u[2 * F + oi];
    dp.x = fma(c, p.x, dp.x); dp.y = fma(c, p.y, dp.y);
    dmn.x = fma(c, m.x, dmn.x); dmn.y = fma(c, m.y, dmn.y);
    dz.x = fma(c, z.x, dz.x); dz.y = fma(c, z.y, dz.y);
  }
  if constexpr (KIND == 1) {
    w[o] = dp;
    w[F + o] = dmn;
    w[2 * F + o] = dz;
    return;
  }
  const cd up = u[o], um = u[F + o], uz = u[2 * F + o];
  // omega+ = i (a/r uz - D1 uz) - b u+ ;  omega- = i (a/r uz + D1 uz) + b u-
  const cd tp = {a * ir * uz.x - dz.x, a * ir * uz.y - dz.y};
  const cd tm = {a * ir * uz.x + dz.x, a * ir * uz.y + dz.y};
  const cd op = {-tp.y - b * up.x, tp.x - b * up.y};
  const cd om = {-tm.y + b * um.x, tm.x + b * um.y};
  // omega_z = -(i/2) [ (D1 + (1+a)/r) u+ - (D1 + (1-a)/r) u- ]
  const cd q = {dp.x + (1.0 + a) * ir * up.x - dmn.x - (1.0 - a) * ir * um.x,
                dp.y + (1.0 + a) * ir * up.y - dmn.y - (1.0 - a) * ir * um.y};
  w[o] = op;
  w[F + o] = om;
  w[2 * F + o] = cd{0.5 * q.y, -0.5 * q.x};
}

template <int KIND>
static hipError_t run_curl(tc_ctx* c, const cd* u, cd* out) {
  const int64_t blocks = (c->d.S + 255) / 256;
  // marching lanes (one per slot) fill fewer than 2 waves per SIMD below
  // 131072 slots per plane: use one thread per point instead
  if (c->d.S < 131072)
    hipLaunchKernelGGL(k_curl_points<KIND>, dim3((unsigned)blocks, (unsigned)c->d.n_r), dim3(256), 0, c->stream,
                       c->rc_dev, c->d, u, out);
  else
    hipLaunchKernelGGL(k_curl<KIND>, dim3((unsigned)blocks), dim3(256), 0, c->stream, c->rc_dev, c->d, u, out);
  return hipGetLastError();
}

hipError_t launch_curl(tc_ctx* c, const cd* u, cd* omega) { return run_curl<0>(c, u, omega); }

hipError_t launch_dr(tc_ctx* c, const cd* u, cd* du) { return run_curl<1>(c, u, du); }

// Scaled packing of u_z and omega_z in the float azimuthal transforms.
#ifndef TC_F32_ZSCALE
#define TC_F32_ZSCALE 1
#endif

// ------------------------------------------------------------------ launch shapes
// z kernels: NF columns per workgroup, TPF threads per column; in-place LDS.
// Swizzled (unpadded) LDS layout in the z kernels (1: FP64 only, 2: both
// precisions): it removes their bank conflicts.  One column tile per
// workgroup.
// Tile width: up to TC_Z_WG threads (twice that for the wide shape below) and TC_Z_LDS_CAP bytes of LDS per workgroup, which at 1536 points
// gives 4 FP64 (8 float) columns, 64 bytes of every row.  Narrower tiles (2 FP64 columns, 32 bytes per row, three
// workgroups per CU) wrote about 1.4x their bytes to HBM and ran at a speed
// that depended on where the buffers' pages landed (k_zinv 16.6-22.9 ms on
// the production planes); 64-byte rows run at 15.1-15.3 ms every time, at
// one workgroup per CU.
#ifndef TC_Z_SWIZZLE
#define TC_Z_SWIZZLE 2
#endif
#ifndef TC_Z_LDS_CAP
#define TC_Z_LDS_CAP 131072
#endif
#ifndef TC_Z_WG
#define TC_Z_WG 512
#endif
template <typename T, int L> struct ZShape {
  static constexpr bool SWZ = (TC_Z_SWIZZLE == 2 || (TC_Z_SWIZZLE == 1 && sizeof(T) == 8)) && L % 16 == 0;
  // 1536 points and above: 256 (FP64) or 128 (float) threads per column,
  // 16 waves in the one workgroup a CU holds; measured 5-10% faster than
  // half as many.  Shorter transforms would leave many of them idle.
  static constexpr bool WIDE = L >= 1536;
  static constexpr int TPF = WIDE ? (sizeof(T) == 8 ? 256 : 128) : L >= 512 ? (sizeof(T) == 8 ? 128 : 64) : (L >= 128 ? 32 : 8);
  static constexpr int LDS_CAP = TC_Z_LDS_CAP;
  static constexpr int NF0 = (WIDE ? 2 * TC_Z_WG : TC_Z_WG) / TPF;
  static constexpr int NF1 = LDS_CAP / (lds_len<L, SWZ>() * (int)sizeof(C2<T>));
  static constexpr int NF = NF0 < NF1 ? NF0 : NF1;
  static_assert(NF >= 1, "transform too long for LDS");
  // Long FP64 transforms exchange one component at a time through LDS (half
  // the bytes), so that two workgroups fit a CU (registers capped for 8
  // waves per SIMD, which these kernels meet without spilling): one
  // workgroup's loads and stores then overlap the other's transform.  At
  // 1536 points this took the inverse pass from 14.4 to 12.7 ms and the
  // forward pass from 7.8 to 6.4 ms on the production planes.  The float
  // kernels (94 and 73 registers) would spill under that cap.
  static constexpr bool SPLIT = WIDE && sizeof(T) == 8;
  static constexpr size_t LDS = (size_t)lds_len<L, SWZ>() * NF * (SPLIT ? sizeof(T) : sizeof(C2<T>));
  static constexpr int WAVES = SPLIT ? 8 : 0;
};
// theta kernel: TPF threads per row, RPB rows per workgroup, the LDS
// exchanges in place (two barriers each).
template <typename T, int L> struct TShape {
  static constexpr int TPF = (L % 6 == 0) ? L / 6 : L / 8;
  static constexpr bool FIREV = false;  // radix order of the inverse transform
  static constexpr int RPB = TPF >= 256 ? 1 : 256 / TPF;
  static constexpr size_t LDS = (size_t)lds_len<L, false>() * RPB * sizeof(C2<T>);
};

// Output weight of the forward z kernel for field fld at azimuthal index n:
// 1 for the forward nonlinear term; for the adjoint transforms the
// Hermitian weights c_n (1 at n = 0, 2 above) on the real-field components
// (fields 4, 5) and c_n / 2 on the complex-pair components (fields 0-3).
__device__ __forceinline__ double z_out_weight(int weights, int fld, int n) {
  if (weights == 0) return 1.0;
  if (fld < 4) return n == 0 ? 0.5 : 1.0;
  return n == 0 ? 1.0 : 2.0;
}

// Tile walk of the z kernels: the grid is 8 ceil(ntiles / 8) workgroups
// and workgroup b takes tile (b % 8) ceil(ntiles / 8) + b / 8, a bijection
// that gives each XCD (workgroups are dispatched round robin over the 8
// XCDs) a contiguous range, so neighbouring column tiles, which share cache
// lines, go through the same L2; tiles past the end belong to padding
// workgroups, which return -1.
__device__ __forceinline__ int single_tile(int ntiles) {
  const int per = (ntiles + 7) / 8;
  const int id = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  return id < ntiles ? id : -1;
}

// ------------------------------------------------------------------ z inverse
template <typename T, int L>
__global__ __launch_bounds__((ZShape<T, L>::NF * ZShape<T, L>::TPF))
__attribute__((amdgpu_waves_per_eu(ZShape<T, L>::WAVES > 0 ? ZShape<T, L>::WAVES : 1))) void k_zinv(Dims d, int plane0,
                                                                                                  int nplanes, ZIo io,
                                                                               C2<T>* __restrict__ inter,
                                                                               const C2<T>* __restrict__ W) {
  using Z = ZShape<T, L>;
  constexpr int NF = Z::NF, TPF = Z::TPF;
  using FI = Fft<T, L, TPF, +1, false, Z::SWZ>;
  extern __shared__ unsigned char lds_raw[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(lds_raw);
  const int tiles = (d.mt + NF - 1) / NF;
  const int ntiles = tiles * io.nfields * nplanes;
  const int f = threadIdx.x % NF, t = threadIdx.x / NF;
  const int h = d.half;
  auto load = [&](int id, cd (&raw)[FI::PER0][FI::R0]) {
    const int tile = id % tiles, rest = id / tiles;
    const int fld = rest % io.nfields, pl = rest / io.nfields;
    const int n = tile * NF + f;
    const cd* src = io.src[fld] + (int64_t)(plane0 + pl) * d.S + n;
#pragma unroll
    for (int k = 0; k < FI::PER0; ++k)
#pragma unroll
      for (int q = 0; q < FI::R0; ++q) {
        const int e = FI::in_index(t, k, q);
        int sl = -1;
        if (e < h) sl = e;
        else if (e > L - h) sl = d.mz - (L - e);
        raw[k][q] = (sl >= 0 && n < d.mt && FI::in_valid(t, k)) ? src[(int64_t)sl * d.mt] : cd{0.0, 0.0};
        if (io.mulb[fld]) {  // i b v, b = l k_z: the axial derivative
          const double bb = (double)(sl < h ? sl : sl - d.mz) * d.kz;
          raw[k][q] = cd{-bb * raw[k][q].y, bb * raw[k][q].x};
        }
      }
  };
  auto transform_store = [&](int id, cd (&raw)[FI::PER0][FI::R0]) {
    typename FI::In v0;
    typename FI::Out vo;
#pragma unroll
    for (int k = 0; k < FI::PER0; ++k)
#pragma unroll
      for (int q = 0; q < FI::R0; ++q) v0[k][q] = C2<T>{T(raw[k][q].x), T(raw[k][q].y)};
    if constexpr (Z::SPLIT) FI::template run_split<NF>(v0, vo, reinterpret_cast<T*>(lds_raw), W, t, f);
    else FI::template run<NF>(v0, vo, buf, buf, W, t, f);
    const int tile = id % tiles, rest = id / tiles;
    const int fld = rest % io.nfields, pl = rest / io.nfields;
    const int n = tile * NF + f;
    if (n < d.mt) {
      C2<T>* dst = inter + ((int64_t)(pl * io.nf_plane + fld) * L) * d.mt + n;
#pragma unroll
      for (int k = 0; k < FI::PERN; ++k)
        if (FI::out_valid(t, k))
#pragma unroll
          for (int s2 = 0; s2 < FI::RN; ++s2) dst[(int64_t)FI::out_index(t, k, s2) * d.mt] = vo[k][s2];
    }
  };
  // per-plane magnitude of two of the input fields (see ZIo::zmax): a wave
  // maximum, then the workgroup's over its waves, then one atomic per
  // workgroup (all the workgroups of a plane update the same word, so
  // fewer atomics contend less); the early returns are uniform over the
  // workgroup, as its barrier needs
  __shared__ float wave_max[(NF * TPF + 63) / 64];
  auto record = [&](int id, const cd (&raw)[FI::PER0][FI::R0]) {
    if (io.zmax == nullptr) return;
    const int rest = id / tiles;
    const int fld = rest % io.nfields, pl = rest / io.nfields;
    const int which = io.zmax_slot[fld];
    if (which < 0) return;
    float m = 0.f;
#pragma unroll
    for (int k = 0; k < FI::PER0; ++k)
#pragma unroll
      for (int q = 0; q < FI::R0; ++q) m = fmaxf(m, (float)fmax(fabs(raw[k][q].x), fabs(raw[k][q].y)));
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) wave_max[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < (int)(blockDim.x / 64); ++w) m = fmaxf(m, wave_max[w]);
      // non-negative floats order as their bit patterns
      atomicMax(io.zmax + ZMAX_WORDS * pl + which, __float_as_uint(m));
    }
  };
  const int id = single_tile(ntiles);
  if (id < 0) return;  // padding workgroup (uniform over the workgroup)
  cd cur[FI::PER0][FI::R0];
  load(id, cur);
  record(id, cur);
  transform_store(id, cur);
}

// ------------------------------------------------------------------ theta pass
template <typename T, int L>
// Register budget of the theta kernel at lengths >= 1024: in double 4 waves
// per SIMD (128 VGPRs), at the cost of a small spill measured faster than
// the unconstrained 3 waves; in float 6 waves.  Shorter rows keep the
// compiler's choice.
#ifndef TC_THETA_WAVES
#define TC_THETA_WAVES 4
#endif
__global__ __launch_bounds__((TShape<T, L>::TPF * TShape<T, L>::RPB))
#if TC_THETA_WAVES
__attribute__((amdgpu_waves_per_eu(L >= 1024 ? (sizeof(T) == 8 ? TC_THETA_WAVES : 6) : 1)))
#endif
void k_theta(Dims d, int nplanes, C2<T>* __restrict__ inter, const C2<T>* __restrict__ W,
             const unsigned int* __restrict__ zmax) {
  using TS = TShape<T, L>;
  constexpr int TPF = TS::TPF, RPB = TS::RPB;
  using FI = Fft<T, L, TPF, +1, TS::FIREV>;
  using FF = Fft<T, L, TPF, -1, !TS::FIREV>;
  static_assert(FI::RN == FF::R0 && FI::PERN == FF::PER0, "mirrored transforms must line up");
  extern __shared__ unsigned char lds_raw[];
  C2<T>* bufa = reinterpret_cast<C2<T>*>(lds_raw);
  C2<T>* bufb = bufa;
  const int f = threadIdx.x % RPB, t = threadIdx.x / RPB;
  const int64_t rows = (int64_t)nplanes * d.pz;
  const int64_t row = (int64_t)blockIdx.x * RPB + f;
  const bool valid = row < rows;
  const int pl = valid ? (int)(row / d.pz) : 0;
  const int z = valid ? (int)(row - (int64_t)pl * d.pz) : 0;
  const int64_t fstride = (int64_t)d.pz * d.mt;  // one field of one plane
  C2<T>* base = inter + (int64_t)pl * 6 * fstride + (int64_t)z * d.mt;
  const int mt = d.mt;

  // spectrum of h_u (which 0), h_omega (1) or g = u_z + i omega_z (2) at
  // azimuthal index e (n = e or e - L)
  // which = 2: g = u_z + i sw omega_z (sw: see below)
  auto spec = [&](int which, int e, T sw) -> C2<T> {
    const C2<T>* A = base + (int64_t)(which == 0 ? 0 : (which == 1 ? 3 : 2)) * fstride;
    const C2<T>* B = base + (int64_t)(which == 0 ? 1 : (which == 1 ? 4 : 5)) * fstride;
    const int nn = (e <= L / 2) ? e : e - L;
    C2<T> v = {T(0), T(0)};
    if (!valid) return v;
    if (which < 2) {
      if (nn > 0 && nn < mt) v = A[nn];
      else if (nn < 0 && -nn < mt) v = cconj(B[-nn]);
      else if (nn == 0) {
        const C2<T> p0 = A[0], m0 = B[0];
        v = {T(0.5) * (p0.x + m0.x), T(0.5) * (p0.y - m0.y)};
      }
    } else {
      if (nn > 0 && nn < mt) {
        const C2<T> x = A[nn], y = B[nn];
        v = {x.x - sw * y.y, x.y + sw * y.x};
      } else if (nn < 0 && -nn < mt) {
        const C2<T> x = cconj(A[-nn]), y = cconj(B[-nn]);
        v = {x.x - sw * y.y, x.y + sw * y.x};
      } else if (nn == 0) {
        v = {A[0].x, sw * B[0].x};
      }
    }
    return v;
  };
  typename FI::In v0;
  typename FI::Out hu, hw, g;
  auto inverse = [&](int which, typename FI::Out& out, T sw) {
#pragma unroll
    for (int k = 0; k < FI::PER0; ++k)
#pragma unroll
      for (int q = 0; q < FI::R0; ++q)
        v0[k][q] = FI::in_valid(t, k) ? spec(which, FI::in_index(t, k, q), sw) : C2<T>{T(0), T(0)};
    FI::template run<RPB>(v0, out, bufa, bufb, W, t, f);
  };
  // g carries u_z and omega_z in one complex transform, whose rounding error
  // delta follows its larger part.  In the products, u_z's error is weighted
  // by |h_omega| and omega_z's by |h_u|, so with g = u_z + i sw omega_z the
  // error of N is about delta (|h_omega| + |h_u| / sw) with delta ~ |u_z| +
  // sw |omega_z|; it is smallest at sw^2 = |u_z| |h_u| / (|omega_z| |h_omega|).
  // In float, sw is that value rounded to a power of two, from the plane's
  // largest coefficients (recorded by the axial inverse kernel), and omega_z
  // is unscaled after the transform (both exact).  In double the unscaled
  // packing costs at most ~1e-13 relative and is kept.
  int ez = 0;
  if constexpr (sizeof(T) == 4) {
    if (zmax != nullptr) {
      float m[ZMAX_WORDS];
      bool ok = true;
#pragma unroll
      for (int w = 0; w < ZMAX_WORDS; ++w) {
        m[w] = __uint_as_float(zmax[ZMAX_WORDS * pl + w]);
        ok = ok && m[w] > 0.f && m[w] < 3e38f;
      }
      if (ok) ez = (ilogbf(m[0]) + ilogbf(m[2]) - ilogbf(m[1]) - ilogbf(m[3])) / 2;
      ez = ez < -40 ? -40 : (ez > 40 ? 40 : ez);
    }
  }
  const T sw = ldexp(T(1), ez), isw = ldexp(T(1), -ez);
  inverse(0, hu, T(1));
  inverse(1, hw, T(1));
  inverse(2, g, sw);
  // pointwise products (the slots hold the same points for all three)
  typename FF::In hn, nz;
#pragma unroll
  for (int k = 0; k < FI::PERN; ++k)
#pragma unroll
    for (int q = 0; q < FI::RN; ++q) {
      const C2<T> a = hu[k][q], w = hw[k][q];
      const T uzv = g[k][q].x, wzv = g[k][q].y * isw;
      hn[k][q] = {uzv * w.y - wzv * a.y, wzv * a.x - uzv * w.x};
      nz[k][q] = {w.x * a.y - w.y * a.x, T(0)};
    }
  typename FF::Out o;
  FF::template run<RPB>(hn, o, bufa, bufb, W, t, f);
  if (valid) {
    C2<T>* Bp = base;
    C2<T>* Bm = base + fstride;
#pragma unroll
    for (int k = 0; k < FF::PERN; ++k)
      if (FF::out_valid(t, k))
#pragma unroll
        for (int s2 = 0; s2 < FF::RN; ++s2) {
          const int e = FF::out_index(t, k, s2);
          if (e < mt) Bp[e] = o[k][s2];
          if (e == 0) Bm[0] = cconj(o[k][s2]);
          else if (L - e < mt) Bm[L - e] = cconj(o[k][s2]);
        }
  }
  FF::template run<RPB>(nz, o, bufa, bufb, W, t, f);
  if (valid) {
    C2<T>* Bz = base + 2 * fstride;
#pragma unroll
    for (int k = 0; k < FF::PERN; ++k)
      if (FF::out_valid(t, k))
#pragma unroll
        for (int s2 = 0; s2 < FF::RN; ++s2) {
          const int e = FF::out_index(t, k, s2);
          if (e < mt) Bz[e] = o[k][s2];
        }
  }
}

// ------------------------------------------------------------------ theta pass, convective form
// The paper's form N = u.grad u (Sec. 3.2, step 1) with the curvature terms
// of eq. NS_cyl, per z-row of a 9-field intermediate: u+, u-, u_z, their
// radial derivatives D1 u+-, D1 u_z, and their axial derivatives i b u+-,
// i b u_z (formed in the axial pass).  Six complex theta transforms carry
// the twelve real fields:
//   h_u = u_r + i u_theta                  spectrum (u+, u-) as a +- pair
//   h_r = d_r u_r + i d_r u_theta          (D1 u+, D1 u-)
//   h_t = (d_theta u_r + i d_theta u_theta)/r   = (i n k_theta / r) times h_u's
//   h_z = d_z u_r + i d_z u_theta          (i b u+, i b u-)
//   g1  = u_z + i d_r u_z,   g2 = d_theta u_z / r + i d_z u_z
// and in physical space, with real u_r, u_theta, u_z,
//   N_r + i N_theta = u_r h_r + u_theta h_t + u_z h_z + i (u_theta / r) h_u
//   (the curvature terms -u_theta^2/r and +u_theta u_r/r), and
//   N_z = u_r d_r u_z + u_theta d_theta u_z / r + u_z d_z u_z.
// The products are accumulated as each inverse transform completes, so at
// most h_u, u_z and the two accumulators are held.  Outputs overwrite
// fields 0-2 of the row, as in the rotational kernel.
// (2 waves per SIMD at lengths >= 1024: the six inverse transforms' held
// fields and accumulators do not fit 3 or 4 waves' budgets without spilling)
#ifndef TC_THETA_CONV_WAVES
#define TC_THETA_CONV_WAVES 2
#endif
template <int L>
__global__ __launch_bounds__((TShape<double, L>::TPF * TShape<double, L>::RPB))
#if TC_THETA_WAVES
__attribute__((amdgpu_waves_per_eu(L >= 1024 ? TC_THETA_CONV_WAVES : 1)))
#endif
void k_theta_conv(Dims d, int plane0, int nplanes, cd* __restrict__ inter, const cd* __restrict__ W,
                  const double* __restrict__ rc) {
  using T = double;
  using TS = TShape<T, L>;
  constexpr int TPF = TS::TPF, RPB = TS::RPB;
  using FI = Fft<T, L, TPF, +1, TS::FIREV>;
  using FF = Fft<T, L, TPF, -1, !TS::FIREV>;
  static_assert(FI::RN == FF::R0 && FI::PERN == FF::PER0, "mirrored transforms must line up");
  extern __shared__ unsigned char lds_raw[];
  cd* bufa = reinterpret_cast<cd*>(lds_raw);
  cd* bufb = bufa;
  const int f = threadIdx.x % RPB, t = threadIdx.x / RPB;
  const int64_t rows = (int64_t)nplanes * d.pz;
  const int64_t row = (int64_t)blockIdx.x * RPB + f;
  const bool valid = row < rows;
  const int pl = valid ? (int)(row / d.pz) : 0;
  const int z = valid ? (int)(row - (int64_t)pl * d.pz) : 0;
  const int64_t fstride = (int64_t)d.pz * d.mt;  // one field of one plane
  cd* base = inter + (int64_t)pl * 9 * fstride + (int64_t)z * d.mt;
  const int mt = d.mt;
  const double ir = rc[(int64_t)(plane0 + pl) * RC_N + RC_IR];
  const double kr = d.kt * ir;  // d_theta / r multiplies mode n by i n k_theta / r

  // +- pair (fields fa, fb): spectrum of v_r + i v_theta at signed index nn
  auto pm = [&](int fa, int fb, int nn) -> cd {
    const cd* A = base + (int64_t)fa * fstride;
    const cd* B = base + (int64_t)fb * fstride;
    if (nn > 0 && nn < mt) return A[nn];
    if (nn < 0 && -nn < mt) return cconj(B[-nn]);
    if (nn == 0) {
      const cd p0 = A[0], m0 = B[0];
      return cd{0.5 * (p0.x + m0.x), 0.5 * (p0.y - m0.y)};
    }
    return cd{0.0, 0.0};
  };
  // two real fields packed as x + i y: x from field fa (times i n k_theta / r
  // when dth), y from field fb
  auto rr = [&](int fa, bool dth, int fb, int nn) -> cd {
    const cd* A = base + (int64_t)fa * fstride;
    const cd* B = base + (int64_t)fb * fstride;
    const int an = nn < 0 ? -nn : nn;
    if (an >= mt) return cd{0.0, 0.0};
    cd x = A[an], y = B[an];
    if (dth) x = cd{-an * kr * x.y, an * kr * x.x};
    if (nn == 0) return cd{x.x, y.x};
    if (nn < 0) {
      x = cconj(x);
      y = cconj(y);
    }
    return cd{x.x - y.y, x.y + y.x};
  };
  // which: 0 h_u, 1 h_r, 2 h_t, 3 h_z, 4 g1, 5 g2
  auto spec = [&](int which, int e) -> cd {
    if (!valid) return cd{0.0, 0.0};
    const int nn = (e <= L / 2) ? e : e - L;
    switch (which) {
      case 0: return pm(0, 1, nn);
      case 1: return pm(3, 4, nn);
      case 2: {
        const cd v = pm(0, 1, nn);
        const double w = nn * kr;
        return cd{-w * v.y, w * v.x};
      }
      case 3: return pm(6, 7, nn);
      case 4: return rr(2, false, 5, nn);
      default: return rr(2, true, 8, nn);
    }
  };
  typename FI::In v0;
  auto inverse = [&](int which, typename FI::Out& out) {
#pragma unroll
    for (int k = 0; k < FI::PER0; ++k)
#pragma unroll
      for (int q = 0; q < FI::R0; ++q)
        v0[k][q] = FI::in_valid(t, k) ? spec(which, FI::in_index(t, k, q)) : cd{0.0, 0.0};
    FI::template run<RPB>(v0, out, bufa, bufb, W, t, f);
  };
  typename FI::Out hu, tmp;
  typename FF::In hn, nz;
  T uz[FI::PERN][FI::RN];
  inverse(0, hu);
  inverse(4, tmp);  // u_z + i d_r u_z
#pragma unroll
  for (int k = 0; k < FI::PERN; ++k)
#pragma unroll
    for (int q = 0; q < FI::RN; ++q) {
      uz[k][q] = tmp[k][q].x;
      nz[k][q] = {hu[k][q].x * tmp[k][q].y, 0.0};
    }
  inverse(1, tmp);  // d_r
#pragma unroll
  for (int k = 0; k < FI::PERN; ++k)
#pragma unroll
    for (int q = 0; q < FI::RN; ++q) hn[k][q] = {hu[k][q].x * tmp[k][q].x, hu[k][q].x * tmp[k][q].y};
  inverse(2, tmp);  // d_theta / r
#pragma unroll
  for (int k = 0; k < FI::PERN; ++k)
#pragma unroll
    for (int q = 0; q < FI::RN; ++q) {
      const T ut = hu[k][q].y;
      hn[k][q] = {fma(ut, tmp[k][q].x, hn[k][q].x), fma(ut, tmp[k][q].y, hn[k][q].y)};
    }
  inverse(3, tmp);  // d_z
#pragma unroll
  for (int k = 0; k < FI::PERN; ++k)
#pragma unroll
    for (int q = 0; q < FI::RN; ++q) {
      const T w = uz[k][q];
      hn[k][q] = {fma(w, tmp[k][q].x, hn[k][q].x), fma(w, tmp[k][q].y, hn[k][q].y)};
    }
  inverse(5, tmp);  // d_theta u_z / r + i d_z u_z
#pragma unroll
  for (int k = 0; k < FI::PERN; ++k)
#pragma unroll
    for (int q = 0; q < FI::RN; ++q) {
      const T ur = hu[k][q].x, ut = hu[k][q].y;
      nz[k][q].x = fma(ut, tmp[k][q].x, fma(uz[k][q], tmp[k][q].y, nz[k][q].x));
      // curvature: i (u_theta / r) h_u
      const T c = ut * ir;
      hn[k][q] = {fma(-c, ut, hn[k][q].x), fma(c, ur, hn[k][q].y)};
    }
  typename FF::Out o;
  FF::template run<RPB>(hn, o, bufa, bufb, W, t, f);
  if (valid) {
    cd* Bp = base;
    cd* Bm = base + fstride;
#pragma unroll
    for (int k = 0; k < FF::PERN; ++k)
      if (FF::out_valid(t, k))
#pragma unroll
        for (int s2 = 0; s2 < FF::RN; ++s2) {
          const int e = FF::out_index(t, k, s2);
          if (e < mt) Bp[e] = o[k][s2];
          if (e == 0) Bm[0] = cconj(o[k][s2]);
          else if (L - e < mt) Bm[L - e] = cconj(o[k][s2]);
        }
  }
  FF::template run<RPB>(nz, o, bufa, bufb, W, t, f);
  if (valid) {
    cd* Bz = base + 2 * fstride;
#pragma unroll
    for (int k = 0; k < FF::PERN; ++k)
      if (FF::out_valid(t, k))
#pragma unroll
        for (int s2 = 0; s2 < FF::RN; ++s2) {
          const int e = FF::out_index(t, k, s2);
          if (e < mt) Bz[e] = o[k][s2];
        }
  }
}

// ------------------------------------------------------------------ theta pass, adjoint
// Transposed nonlinear term (used by the discrete adjoint step), per z-row
// of the transform-layout buffer holding 9 fields per plane: the forward
// fields (u+, u-, u_z, omega+, omega-, omega_z) and the cotangent of N
// (N+, N-, N_z) after the axial inverse transform.  The transpose of the
// forward transform (1/P, truncation, Hermitian half spectrum) is an
// inverse transform of the cotangent with weight 1 on every stored mode:
// h_g = g_r + i g_theta has spectrum N+ (n > 0), conj(N-(|n|)) (n < 0),
// N+ + conj(N-) (n = 0), and g_z is the real part of the one-sided sum of
// N_z.  Then omega_bar = u x g and u_bar = g x omega pointwise, and the
// forward transforms of u_bar_r + i u_bar_theta, omega_bar_r + i
// omega_bar_theta and u_bar_z + i omega_bar_z give (after the axial pass with
// Hermitian weights) the cotangents of u+-, omega+-, u_z, omega_z.  The six
// results overwrite fields of the row that have been consumed: u_bar+- go
// to fields 6, 7 (see adjoint_field_map), omega_bar+- to 2, 3 and u_bar_z,
// omega_bar_z to 4, 5.  The transforms are staged so that few spectra are
// held at once (3 waves per SIMD at the long lengths: 78.8 ms against 82.9
// ms for the adjoint step at scale with all five inverse spectra held).
template <typename T, int L>
#ifndef TC_THETA_ADJ_WAVES
#define TC_THETA_ADJ_WAVES 3
#endif
__global__ __launch_bounds__((TShape<T, L>::TPF * TShape<T, L>::RPB))
__attribute__((amdgpu_waves_per_eu(L >= 1024 ? TC_THETA_ADJ_WAVES : 1))) void k_theta_adj(Dims d, int nplanes,
                                                                                     C2<T>* __restrict__ inter,
                                                                                     const C2<T>* __restrict__ W) {
  using TS = TShape<T, L>;
  constexpr int TPF = TS::TPF, RPB = TS::RPB;
  using FI = Fft<T, L, TPF, +1, TS::FIREV>;
  using FF = Fft<T, L, TPF, -1, !TS::FIREV>;
  extern __shared__ unsigned char lds_raw[];
  C2<T>* bufa = reinterpret_cast<C2<T>*>(lds_raw);
  C2<T>* bufb = bufa;
  const int f = threadIdx.x % RPB, t = threadIdx.x / RPB;
  const int64_t rows = (int64_t)nplanes * d.pz;
  const int64_t row = (int64_t)blockIdx.x * RPB + f;
  const bool valid = row < rows;
  const int pl = valid ? (int)(row / d.pz) : 0;
  const int z = valid ? (int)(row - (int64_t)pl * d.pz) : 0;
  const int64_t fstride = (int64_t)d.pz * d.mt;
  C2<T>* base = inter + (int64_t)pl * 9 * fstride + (int64_t)z * d.mt;
  const int mt = d.mt;
  auto fld = [&](int k) { return base + (int64_t)k * fstride; };
  // mode: 0 pair (n = 0 averaged), 1 packed real pair, 2 pair (n = 0 summed), 3 one-sided
  auto spec = [&](int mode, const C2<T>* A, const C2<T>* B, int e) -> C2<T> {
    const int nn = (e <= L / 2) ? e : e - L;
    C2<T> v = {T(0), T(0)};
    if (!valid) return v;
    if (mode == 0 || mode == 2) {
      if (nn > 0 && nn < mt) v = A[nn];
      else if (nn < 0 && -nn < mt) v = cconj(B[-nn]);
      else if (nn == 0) {
        const C2<T> p0 = A[0], m0 = B[0];
        const T w = mode == 0 ? T(0.5) : T(1);
        v = {w * (p0.x + m0.x), w * (p0.y - m0.y)};
      }
    } else if (mode == 1) {
      if (nn > 0 && nn < mt) {
        const C2<T> x = A[nn], y = B[nn];
        v = {x.x - y.y, x.y + y.x};
      } else if (nn < 0 && -nn < mt) {
        const C2<T> x = cconj(A[-nn]), y = cconj(B[-nn]);
        v = {x.x - y.y, x.y + y.x};
      } else if (nn == 0) {
        v = {A[0].x, B[0].x};
      }
    } else {
      if (nn >= 0 && nn < mt) v = A[nn];
    }
    return v;
  };
  typename FI::In v0;
  auto inverse = [&](int mode, const C2<T>* A, const C2<T>* B, typename FI::Out& out) {
#pragma unroll
    for (int k = 0; k < FI::PER0; ++k)
#pragma unroll
      for (int q = 0; q < FI::R0; ++q)
        v0[k][q] = FI::in_valid(t, k) ? spec(mode, A, B, FI::in_index(t, k, q)) : C2<T>{T(0), T(0)};
    FI::template run<RPB>(v0, out, bufa, bufb, W, t, f);
  };
  // The cotangent transforms first, then omega (whose products are
  // finished and transformed at once, their outputs going to the consumed
  // fields 6, 7), then u; at most h_g, g_z, u_z and one partial product
  // are held between transforms.
  typename FI::Out hg, tmp;
  T gzr[FI::PERN][FI::RN], uzr[FI::PERN][FI::RN], wzr[FI::PERN][FI::RN], a3x[FI::PERN][FI::RN];
  inverse(2, fld(6), fld(7), hg);
  inverse(3, fld(8), fld(8), tmp);
#pragma unroll
  for (int k = 0; k < FI::PERN; ++k)
#pragma unroll
    for (int q = 0; q < FI::RN; ++q) gzr[k][q] = tmp[k][q].x;
  inverse(1, fld(2), fld(5), tmp);  // u_z + i omega_z
#pragma unroll
  for (int k = 0; k < FI::PERN; ++k)
#pragma unroll
    for (int q = 0; q < FI::RN; ++q) {
      uzr[k][q] = tmp[k][q].x;
      wzr[k][q] = tmp[k][q].y;
    }
  inverse(0, fld(3), fld(4), tmp);  // omega_r + i omega_theta
  typename FF::In a;
#pragma unroll
  for (int k = 0; k < FI::PERN; ++k)
#pragma unroll
    for (int q = 0; q < FI::RN; ++q) {
      const T wr = tmp[k][q].x, wt = tmp[k][q].y, wz = wzr[k][q];
      const T gr = hg[k][q].x, gt = hg[k][q].y, gzv = gzr[k][q];
      // u_bar = g x omega; the omega part of omega_bar_z's partner below
      a[k][q] = {gt * wz - gzv * wt, gzv * wr - gr * wz};
      a3x[k][q] = gr * wt - gt * wr;
    }
  typename FF::Out o;
  auto store_pair = [&](int fa, int fb) {
    if (!valid) return;
    C2<T>* Bp = fld(fa);
    C2<T>* Bm = fld(fb);
#pragma unroll
    for (int k = 0; k < FF::PERN; ++k)
      if (FF::out_valid(t, k))
#pragma unroll
        for (int s2 = 0; s2 < FF::RN; ++s2) {
          const int e = FF::out_index(t, k, s2);
          if (e < mt) Bp[e] = o[k][s2];
          if (e == 0) Bm[0] = cconj(o[k][s2]);
          else if (L - e < mt) Bm[L - e] = cconj(o[k][s2]);
        }
  };
  FF::template run<RPB>(a, o, bufa, bufb, W, t, f);
  store_pair(6, 7);
  inverse(0, fld(0), fld(1), tmp);  // u_r + i u_theta
  typename FF::In a3;
#pragma unroll
  for (int k = 0; k < FI::PERN; ++k)
#pragma unroll
    for (int q = 0; q < FI::RN; ++q) {
      const T ur = tmp[k][q].x, ut = tmp[k][q].y, uz = uzr[k][q];
      const T gr = hg[k][q].x, gt = hg[k][q].y, gzv = gzr[k][q];
      // omega_bar = u x g
      a[k][q] = {ut * gzv - uz * gt, uz * gr - ur * gzv};
      a3[k][q] = {a3x[k][q], ur * gt - ut * gr};
    }
  FF::template run<RPB>(a, o, bufa, bufb, W, t, f);
  store_pair(2, 3);
  FF::template run<RPB>(a3, o, bufa, bufb, W, t, f);
  // separate the packed real fields: X(n) = (G(n) + conj G(-n))/2, Y(n) = (G(n) - conj G(-n))/(2i)
  // G(n) and G(-n) sit in different threads: go through LDS
#pragma unroll
  for (int k = 0; k < FF::PERN; ++k)
    if (FF::out_valid(t, k))
#pragma unroll
      for (int s2 = 0; s2 < FF::RN; ++s2) bufa[lds_slot<L, false>(FF::out_index(t, k, s2)) * RPB + f] = o[k][s2];
  __syncthreads();
  if (valid) {
    C2<T>* X = fld(4);
    C2<T>* Y = fld(5);
    for (int nn = t; nn < mt; nn += TPF) {
      const C2<T> gp = bufa[lds_slot<L, false>(nn) * RPB + f];
      const C2<T> gm = cconj(bufa[lds_slot<L, false>((L - nn) % L) * RPB + f]);
      X[nn] = {T(0.5) * (gp.x + gm.x), T(0.5) * (gp.y + gm.y)};
      Y[nn] = {T(0.5) * (gp.y - gm.y), T(-0.5) * (gp.x - gm.x)};
    }
  }
}

// ------------------------------------------------------------------ z forward
template <typename T, int L>
__global__ __launch_bounds__((ZShape<T, L>::NF * ZShape<T, L>::TPF))
__attribute__((amdgpu_waves_per_eu(ZShape<T, L>::WAVES > 0 ? ZShape<T, L>::WAVES : 1))) void k_zfwd(Dims d, int plane0,
                                                                                                  int nplanes, ZIo io,
                                                                               const C2<T>* __restrict__ inter,
                                                                               const C2<T>* __restrict__ W) {
  using Z = ZShape<T, L>;
  constexpr int NF = Z::NF, TPF = Z::TPF;
  using FF = Fft<T, L, TPF, -1, false, Z::SWZ>;
  extern __shared__ unsigned char lds_raw[];
  C2<T>* buf = reinterpret_cast<C2<T>*>(lds_raw);
  const int tiles = (d.mt + NF - 1) / NF;
  const int ntiles = tiles * io.nfields * nplanes;
  const int f = threadIdx.x % NF, t = threadIdx.x / NF;
  const int h = d.half;
  // per-plane magnitude words of the batch (see ZIo::zmax), read by the
  // azimuthal pass that ran before this one: zero again for the next batch
  if (io.zmax != nullptr && blockIdx.x == 0)
    for (int i = threadIdx.x; i < ZMAX_WORDS * nplanes; i += blockDim.x) io.zmax[i] = 0u;
  auto load = [&](int id, typename FF::In& v) {
    const int tile = id % tiles, rest = id / tiles;
    const int fld = rest % io.nfields, pl = rest / io.nfields;
    const int n = tile * NF + f;
    const int sf = io.use_map ? io.src_field[fld] : fld;
    const C2<T>* src = inter + ((int64_t)(pl * io.nf_plane + sf) * L) * d.mt + n;
#pragma unroll
    for (int k = 0; k < FF::PER0; ++k)
#pragma unroll
      for (int q = 0; q < FF::R0; ++q)
        v[k][q] = (n < d.mt && FF::in_valid(t, k)) ? src[(int64_t)FF::in_index(t, k, q) * d.mt] : C2<T>{T(0), T(0)};
  };
  auto transform_store = [&](int id, typename FF::In& cur) {
    typename FF::Out vo;
    if constexpr (Z::SPLIT) FF::template run_split<NF>(cur, vo, reinterpret_cast<T*>(lds_raw), W, t, f);
    else FF::template run<NF>(cur, vo, buf, buf, W, t, f);
    const int tile = id % tiles, rest = id / tiles;
    const int fld = rest % io.nfields, pl = rest / io.nfields;
    const int n = tile * NF + f;
    if (n < d.mt) {
      cd* dst = io.dst[fld] + (int64_t)(plane0 + pl) * d.S + n;
      const double scale = io.scale * z_out_weight(io.weights, fld, n);
#pragma unroll
      for (int k = 0; k < FF::PERN; ++k)
        if (FF::out_valid(t, k))
#pragma unroll
          for (int s2 = 0; s2 < FF::RN; ++s2) {
            const int e = FF::out_index(t, k, s2);
            int sl = -1;
            if (e < h) sl = e;
            else if (e > L - h) sl = d.mz - (L - e);
            if (sl >= 0) {
              const C2<T> x = vo[k][s2];
              dst[(int64_t)sl * d.mt] = cd{double(x.x) * scale, double(x.y) * scale};
            }
          }
      if (t == 0) dst[(int64_t)h * d.mt] = cd{0.0, 0.0};
    }
  };
  const int id = single_tile(ntiles);
  if (id < 0) return;  // padding workgroup (uniform over the workgroup)
  typename FF::In cur;
  load(id, cur);
  transform_store(id, cur);
}

// ------------------------------------------------------------------ dispatch
// Supported transform lengths: 2^k, 3 2^k, 9 2^k, 5 2^k and 15 2^k from 16 to
// 2048 (radices 8, 4, 2, 3, 5), among them the paper's 320, 384, 640 and the
// dealiased 480, 960 of its 320- and 640-point axial grids.
#define TC_FFT_LENGTHS(X)                                                                                        \
  X(16) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(120) X(128) X(144) X(160) X(192) X(240) X(256) X(288) X(320) \
  X(384) X(480) X(512) X(576) X(640) X(768) X(960) X(1024) X(1152) X(1280) X(1536) X(1920) X(2048)

bool fft_length_supported(int L) {
#define TC_CASE(LL) if (L == LL) return true;
  TC_FFT_LENGTHS(TC_CASE)
#undef TC_CASE
  return false;
}

int inter_fields(const tc_ctx* c) { return c->d.form == TC_CONVECTIVE ? 9 : 6; }

size_t inter_bytes_per_plane(const tc_ctx* c) {
  const size_t el = (c->g.precision == TC_FP32_BULK) ? sizeof(cf) : sizeof(cd);
  return (size_t)inter_fields(c) * c->d.pz * c->d.mt * el;
}

// Workgroups of a z kernel: one per tile, padded to a multiple of 8 (see
// single_tile).
static unsigned z_blocks(int64_t ntiles) { return (unsigned)(8 * ((ntiles + 7) / 8)); }

template <typename T, int L>
static hipError_t run_zinv(tc_ctx* c, int plane0, int np, const ZIo& io, void* inter, const C2<T>* W) {
  using Z = ZShape<T, L>;
  const size_t lds = Z::LDS;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_zinv<T, L>), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    attr = true;
  }
  const int tiles = (c->d.mt + Z::NF - 1) / Z::NF;
  const unsigned blocks = z_blocks((int64_t)np * io.nfields * tiles);
  hipLaunchKernelGGL((k_zinv<T, L>), dim3(blocks), dim3(Z::NF * Z::TPF), lds, c->stream, c->d, plane0, np, io,
                     reinterpret_cast<C2<T>*>(inter), W);
  return hipGetLastError();
}

template <typename T, int L>
static hipError_t run_theta(tc_ctx* c, int np, const C2<T>* W) {
  using TS = TShape<T, L>;
  const size_t lds = TS::LDS;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_theta<T, L>), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    attr = true;
  }
  const int64_t rows = (int64_t)np * c->d.pz;
  const unsigned blocks = (unsigned)((rows + TS::RPB - 1) / TS::RPB);
  hipLaunchKernelGGL((k_theta<T, L>), dim3(blocks), dim3(TS::TPF * TS::RPB), lds, c->stream, c->d, np,
                     reinterpret_cast<C2<T>*>(c->inter), W, TC_F32_ZSCALE ? (const unsigned int*)c->zmax : nullptr);
  return hipGetLastError();
}

template <typename T, int L>
static hipError_t run_zfwd(tc_ctx* c, int plane0, int np, const ZIo& io, const void* inter, const C2<T>* W) {
  using Z = ZShape<T, L>;
  const size_t lds = Z::LDS;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_zfwd<T, L>), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    attr = true;
  }
  const int tiles = (c->d.mt + Z::NF - 1) / Z::NF;
  const unsigned blocks = z_blocks((int64_t)np * io.nfields * tiles);
  hipLaunchKernelGGL((k_zfwd<T, L>), dim3(blocks), dim3(Z::NF * Z::TPF), lds, c->stream, c->d, plane0, np, io,
                     reinterpret_cast<const C2<T>*>(inter), W);
  return hipGetLastError();
}

hipError_t launch_zinv(tc_ctx* c, int plane0, int np, const cd* u, const cd* om) {
  ZIo io{};
  for (int k = 0; k < 3; ++k) {
    io.src[k] = u + k * c->d.F;
    io.src[3 + k] = om + k * c->d.F;
  }
  io.nfields = 6;
  io.nf_plane = 6;
  const bool f32 = c->g.precision == TC_FP32_BULK;
  if (f32 && TC_F32_ZSCALE) {
    // per-plane magnitudes of u_z, omega_z, u+- and omega+-, for the scaled
    // packing of the azimuthal float transforms
    io.zmax = c->zmax;
    const int slot[6] = {2, 2, 0, 3, 3, 1};
    for (int k = 0; k < 9; ++k) io.zmax_slot[k] = k < 6 ? slot[k] : -1;
    // (the words start at zero: cleared at tc_init and by the forward axial
    // pass that follows each azimuthal float pass)
  }
  return launch_zinv_io(c, plane0, np, io, c->inter, f32);
}

hipError_t launch_zinv_io(tc_ctx* c, int plane0, int np, const ZIo& io, void* inter, bool f32) {
#define TC_CASE(LL)                                                                        \
  if (c->d.pz == LL) return f32 ? run_zinv<float, LL>(c, plane0, np, io, inter, c->twf_z) \
                                : run_zinv<double, LL>(c, plane0, np, io, inter, c->tw_z);
  TC_FFT_LENGTHS(TC_CASE)
#undef TC_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_theta(tc_ctx* c, int np) {
  const bool f32 = c->g.precision == TC_FP32_BULK;
#define TC_CASE(LL) \
  if (c->d.pt == LL) return f32 ? run_theta<float, LL>(c, np, c->twf_t) : run_theta<double, LL>(c, np, c->tw_t);
  TC_FFT_LENGTHS(TC_CASE)
#undef TC_CASE
  return hipErrorInvalidValue;
}

template <int L>
static hipError_t run_theta_adj(tc_ctx* c, int np, void* inter) {
  using TS = TShape<double, L>;
  const size_t lds = TS::LDS;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_theta_adj<double, L>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr = true;
  }
  const int64_t rows = (int64_t)np * c->d.pz;
  const unsigned blocks = (unsigned)((rows + TS::RPB - 1) / TS::RPB);
  hipLaunchKernelGGL((k_theta_adj<double, L>), dim3(blocks), dim3(TS::TPF * TS::RPB), lds, c->stream, c->d, np,
                     reinterpret_cast<cd*>(inter), c->tw_t);
  return hipGetLastError();
}

void adjoint_field_map(ZIo& zo) {
  const int where[6] = {6, 7, 2, 3, 4, 5};
  zo.use_map = 1;
  for (int k = 0; k < 6; ++k) zo.src_field[k] = where[k];
}

hipError_t launch_theta_adj(tc_ctx* c, int np, void* inter) {
#define TC_CASE(LL) \
  if (c->d.pt == LL) return run_theta_adj<LL>(c, np, inter);
  TC_FFT_LENGTHS(TC_CASE)
#undef TC_CASE
  return hipErrorInvalidValue;
}

template <int L>
static hipError_t run_theta_conv(tc_ctx* c, int plane0, int np) {
  using TS = TShape<double, L>;
  const size_t lds = TS::LDS;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_theta_conv<L>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr = true;
  }
  const int64_t rows = (int64_t)np * c->d.pz;
  const unsigned blocks = (unsigned)((rows + TS::RPB - 1) / TS::RPB);
  hipLaunchKernelGGL((k_theta_conv<L>), dim3(blocks), dim3(TS::TPF * TS::RPB), lds, c->stream, c->d, plane0, np,
                     reinterpret_cast<cd*>(c->inter), c->tw_t, c->rc_dev);
  return hipGetLastError();
}

hipError_t launch_theta_conv(tc_ctx* c, int plane0, int np) {
#define TC_CASE(LL) \
  if (c->d.pt == LL) return run_theta_conv<LL>(c, plane0, np);
  TC_FFT_LENGTHS(TC_CASE)
#undef TC_CASE
  return hipErrorInvalidValue;
}

// Convective form: u+-, u_z, their radial derivatives and (multiplied by
// i b in the load) their axial derivatives, 9 fields per plane.
hipError_t launch_zinv_conv(tc_ctx* c, int plane0, int np, const cd* u, const cd* du) {
  ZIo io{};
  for (int k = 0; k < 3; ++k) {
    io.src[k] = u + k * c->d.F;
    io.src[3 + k] = du + k * c->d.F;
    io.src[6 + k] = u + k * c->d.F;
    io.mulb[6 + k] = 1;
  }
  for (int k = 0; k < 9; ++k) io.zmax_slot[k] = -1;
  io.nfields = 9;
  io.nf_plane = 9;
  return launch_zinv_io(c, plane0, np, io, c->inter, false);
}

hipError_t launch_zfwd(tc_ctx* c, int plane0, int np, cd* N) {
  ZIo io{};
  for (int k = 0; k < 3; ++k) io.dst[k] = N + k * c->d.F;
  io.nfields = 3;
  io.nf_plane = inter_fields(c);
  io.scale = 1.0 / ((double)c->d.pt * (double)c->d.pz);
  io.weights = 0;
  const bool f32 = c->g.precision == TC_FP32_BULK;
  // the per-plane magnitudes the azimuthal float pass has just used are
  // cleared by this pass for the next axial inverse pass
  if (f32 && TC_F32_ZSCALE) io.zmax = c->zmax;
  return launch_zfwd_io(c, plane0, np, io, c->inter, f32);
}

hipError_t launch_zfwd_io(tc_ctx* c, int plane0, int np, const ZIo& io, const void* inter, bool f32) {
#define TC_CASE(LL)                                                                       \
  if (c->d.pz == LL) return f32 ? run_zfwd<float, LL>(c, plane0, np, io, inter, c->twf_z) \
                                : run_zfwd<double, LL>(c, plane0, np, io, inter, c->tw_z);
  TC_FFT_LENGTHS(TC_CASE)
#undef TC_CASE
  return hipErrorInvalidValue;
}

}  // namespace tc
