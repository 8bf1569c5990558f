// Predictor-corrector of one step with every radial line held on chip
// (Sec. 3.2, steps 2-5): the solves, stencils and update of the four-sweep
// kernels of tc_solve.hip, for grids of n_r = 8 LPS radial nodes (LPS, the
// lanes per slot, a power of two up to 16).  On such grids the four-sweep
// kernels have too few lanes (one per distinct mode) to hide the latency
// of their radial chains; here a slot's line is spread over LPS lanes.
//
// Work decomposition: LPS lanes per axial slot of a distinct mode (|l|, n),
// 64 / LPS slots of consecutive distinct modes per wave.  Lane k of a slot
// holds rows 8k .. 8k+7 of every radial field of that slot, in registers
// and LDS, so the step's intermediates (Ne, p*, the Helmholtz right-hand
// sides, u*, phi) never leave the chip: the kernel reads u^i, u^{i-1}, N^i,
// N^{i-1} and the factors once and writes u^{i+1}, p and, when asked, the
// curl of u^{i+1} that the next step's nonlinear term needs.  A load of
// one row across a wave reads 64 / LPS consecutive slots: whole cache
// lines from LPS = 8 down.
//
// Banded substitutions across lanes: a sweep of the unpivoted LU factors is
// a linear recurrence of order 4 along the rows (each output depends on the
// 4 previous ones in the sweep's order).  Each lane runs the recurrence over
// its 8 rows from a zero incoming state, which gives the affine map (T, g)
// from the 4 values it receives to the 4 it passes on; a Kogge-Stone scan of
// these maps over the slot's lanes (log2 LPS levels of shuffles) gives
// every lane its true incoming state, and the lane runs its rows again from
// it.  The rows a lane finally computes are the sequential sweep's, up to
// the rounding of the incoming state.
//
// Stencils (D1 over +-4 rows) take their 4 halo rows from the neighbouring
// lanes by shuffles; the per-row stencil weights sit in LDS.
//
// The factors are a second, lane-contiguous copy of the ones the other
// solves use (flin, tc_internal.h).  Tiles of 16 waves' distinct modes x 2
// axial signs (8 workgroups) are dispatched consecutively to one XCD, so
// the two slots of a mode, which read the same factors, go through the
// same L2.
#include "tc_internal.h"

namespace tc {
namespace {

constexpr int RPL = LINE_RPL;
constexpr int NLANE = 64;  // lanes per wave
static_assert(RPL >= HW + 1, "the wall terms of a line must lie within one lane");
// per-lane stencil table in LDS: W1 (9 weights) and 1/r for each row
constexpr int TAB_F = NB9 + 1;
constexpr int TAB_IR = NB9;
// waves per workgroup; LDS per wave for the three velocity fields
constexpr int WAVES = 4;

typedef double dbl2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ cd z0() { return cd{0.0, 0.0}; }
__device__ __forceinline__ cd fmac(cd acc, double w, cd v) { return cd{fma(w, v.x, acc.x), fma(w, v.y, acc.y)}; }
__device__ __forceinline__ cd nfmac(cd acc, double w, cd v) { return cd{fma(-w, v.x, acc.x), fma(-w, v.y, acc.y)}; }
__device__ __forceinline__ cd scl(cd v, double w) { return cd{v.x * w, v.y * w}; }
// i * w * v
__device__ __forceinline__ cd imul(cd v, double w) { return cd{-w * v.y, w * v.x}; }
__device__ __forceinline__ cd shfl_c(cd v, int src) { return cd{__shfl(v.x, src, NLANE), __shfl(v.y, src, NLANE)}; }

// Window of a field around the lane's rows: w[i] holds row 8k - 4 + i of
// the lane's slot (zero outside the line); ch = k, the lane's place in it.
template <int LPS>
__device__ __forceinline__ void halo(const cd (&x)[RPL], cd (&w)[RPL + 2 * HW], int lane, int ch) {
#pragma unroll
  for (int i = 0; i < HW; ++i) {
    const cd lo = shfl_c(x[RPL - HW + i], (lane - 1) & (NLANE - 1));
    const cd hi = shfl_c(x[i], (lane + 1) & (NLANE - 1));
    w[i] = ch == 0 ? z0() : lo;
    w[RPL + HW + i] = ch == LPS - 1 ? z0() : hi;
  }
#pragma unroll
  for (int r = 0; r < RPL; ++r) w[HW + r] = x[r];
}

// D1 of a windowed field at the lane's row r
template <int LPS>
__device__ __forceinline__ cd d1_at(const double* tab, int ch, int r, const cd (&w)[RPL + 2 * HW]) {
  cd s = z0();
#pragma unroll
  for (int m = 0; m < NB9; ++m) s = fmac(s, tab[(r * TAB_F + m) * LPS + ch], w[r + m]);
  return s;
}

// Factor loads (flin layout, tc_internal.h).  First part: the first-sweep
// multipliers m[r][c]; second part: the inverse pivot s[r] and the
// second-sweep coefficients m[r][c].
template <int LPS>
__device__ __forceinline__ void load_first(const double* f, double (&m)[RPL][4]) {
#pragma unroll
  for (int q = 0; q < LINE_Q1; ++q) {
    const dbl2 v = *reinterpret_cast<const dbl2*>(f + (int64_t)q * 2 * LPS);
    const int e = 2 * q;
    m[e / 4][e % 4] = v.x;
    m[(e + 1) / 4][(e + 1) % 4] = v.y;
  }
}
template <int LPS>
__device__ __forceinline__ void load_second(const double* f, double (&s)[RPL], double (&m)[RPL][4]) {
#pragma unroll
  for (int q = LINE_Q1; q < LINE_Q; ++q) {
    const dbl2 v = *reinterpret_cast<const dbl2*>(f + (int64_t)q * 2 * LPS);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = 2 * (q - LINE_Q1) + h;
      const int r = e / 5, cc = e % 5;
      const double x = h ? v.y : v.x;
      if (cc == 0) s[r] = x;
      else m[r][cc - 1] = x;
    }
  }
}

// One substitution over the line.  In processing order (rows ascending when
// ASC, else descending) y_i = (f_i - sum_{c<4} m_i[c] y_{i-1-c}) s_i, with
// s_i = 1 unless SCALED; f (indexed by row) is overwritten with y.
template <int LPS, bool ASC, bool SCALED>
__device__ __forceinline__ void line_solve(const double (&m)[RPL][4], const double (&s)[RPL], cd (&f)[RPL], int lane,
                                           int ch) {
  // local pass from a zero incoming state: g = last 4 outputs (newest
  // first), T[i][e] = their dependence on incoming value e
  cd g[4] = {z0(), z0(), z0(), z0()};
  double T[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) T[i][e] = (i == e) ? 1.0 : 0.0;
#pragma unroll
  for (int p = 0; p < RPL; ++p) {
    const int r = ASC ? p : RPL - 1 - p;
    cd v = f[r];
    double w[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      v = nfmac(v, m[r][c], g[c]);
#pragma unroll
      for (int e = 0; e < 4; ++e) w[e] = fma(-m[r][c], T[c][e], w[e]);
    }
    if (SCALED) {
      v = scl(v, s[r]);
#pragma unroll
      for (int e = 0; e < 4; ++e) w[e] *= s[r];
    }
#pragma unroll
    for (int c = 3; c >= 1; --c) {
      g[c] = g[c - 1];
#pragma unroll
      for (int e = 0; e < 4; ++e) T[c][e] = T[c - 1][e];
    }
    g[0] = v;
#pragma unroll
    for (int e = 0; e < 4; ++e) T[0][e] = w[e];
  }
  // inclusive scan of the maps in processing order over the slot's lanes:
  // after the level of distance d a lane holds the composition over itself
  // and the 2d - 1 lanes before it
#pragma unroll
  for (int dist = 1; dist < LPS; dist *= 2) {
    const int src = (ASC ? lane - dist : lane + dist) & (NLANE - 1);
    const bool ok = ASC ? (ch >= dist) : (ch + dist < LPS);
    const bool last = 2 * dist == LPS;
    cd gs[4];
    double Ts[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) gs[i] = shfl_c(g[i], src);
    if (!last) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) Ts[i][e] = __shfl(T[i][e], src, NLANE);
    }
    if (ok) {
      cd gn[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        gn[i] = g[i];
#pragma unroll
        for (int c = 0; c < 4; ++c) gn[i] = fmac(gn[i], T[i][c], gs[c]);
      }
      if (!last) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          double t[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            t[e] = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) t[e] = fma(T[i][c], Ts[c][e], t[e]);
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) T[i][e] = t[e];
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) g[i] = gn[i];
    }
  }
  // incoming state: the outputs of the preceding lane; then the lane's rows
  const int pred = (ASC ? lane - 1 : lane + 1) & (NLANE - 1);
  const bool first = ASC ? ch == 0 : ch == LPS - 1;
  cd y[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const cd t = shfl_c(g[i], pred);
    y[i] = first ? z0() : t;
  }
#pragma unroll
  for (int p = 0; p < RPL; ++p) {
    const int r = ASC ? p : RPL - 1 - p;
    cd v = f[r];
#pragma unroll
    for (int c = 0; c < 4; ++c) v = nfmac(v, m[r][c], y[c]);
    if (SCALED) v = scl(v, s[r]);
#pragma unroll
    for (int c = 3; c >= 1; --c) y[c] = y[c - 1];
    y[0] = v;
    f[r] = v;
  }
}

// Solve with operator op: LU (P, ascending) or UL (H, descending) factors.
template <int LPS, bool LU>
__device__ __forceinline__ void line_op_solve(const double* fl, cd (&f)[RPL], int lane, int ch) {
  double m[RPL][4], s[RPL];
  load_first<LPS>(fl, m);
  line_solve<LPS, LU, false>(m, s, f, lane, ch);
  __builtin_amdgcn_sched_barrier(0);
  load_second<LPS>(fl, s, m);
  line_solve<LPS, !LU, true>(m, s, f, lane, ch);
}

}  // namespace

template <int LPS, bool FUSE>
__global__ __launch_bounds__(WAVES * NLANE) void k_pcl(const double* __restrict__ rc, const double* __restrict__ flin,
                                                      Dims d, const cd* __restrict__ u, const cd* up,
                                                      const cd* __restrict__ N, const cd* __restrict__ Np, cd* un,
                                                      cd* p, int want_p, cd* omg, int ntile, int per) {
  constexpr int SPW = NLANE / LPS;  // slots (distinct modes) per wave
  __shared__ double tab[RPL * TAB_F * LPS];
  // the three velocity fields of each wave's lines (Helmholtz right-hand
  // sides, then u*, then u^{i+1}); each lane touches only its own entries
  __shared__ cd vel[WAVES * 3 * RPL * NLANE];
  const int lane = threadIdx.x % NLANE, wv = threadIdx.x / NLANE;
  const int seg = lane / LPS, ch = lane % LPS;
  for (int i = threadIdx.x; i < RPL * TAB_F * LPS; i += blockDim.x) {
    const int k = i % LPS, rf = i / LPS, r = rf / TAB_F, f = rf % TAB_F;
    const double* R = rc + (int64_t)(RPL * k + r) * RC_N;
    tab[i] = f < NB9 ? R[RC_W1 + f] : R[RC_IR];
  }
  __syncthreads();
  // tile t: 16 SPW distinct modes x 2 signs = 8 workgroups, the x-th XCD
  // taking tiles x per .. (x + 1) per - 1 in order
  const int x = blockIdx.x % 8, rr = blockIdx.x / 8;
  const int t = x * per + rr / 8, q = rr % 8;
  if (t >= ntile) return;
  const int sign = q & 1;
  const int dm = ((t * 4 + (q >> 1)) * WAVES + wv) * SPW + seg;
  const bool active = dm < d.ndm;
  if (__ballot(active) == 0) return;
  const int dmc = active ? dm : d.ndm - 1;
  const int labs = dmc / d.mt, n = dmc - labs * d.mt;
  // a lane of sign -1 at |l| = 0 keeps the empty axial slot (l = -m_z/2) of
  // its n at zero; it and the lanes past the last mode compute on slot 0's
  // data (the wave's shuffles need every lane) and store nothing else
  const bool nyq = active && sign == 1 && labs == 0;
  const bool reg = active && !nyq;
  const int M = d.n_r - 1;
  const int64_t F = d.F, S = d.S;
  const int j0 = RPL * ch;
  if (nyq) {
    const int64_t on = (int64_t)d.nyq * d.mt + n;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int64_t oj = (int64_t)(j0 + r) * S + on;
      un[oj] = z0();
      un[F + oj] = z0();
      un[2 * F + oj] = z0();
      if (want_p) p[oj] = z0();
      if (FUSE) {
        omg[oj] = z0();
        omg[F + oj] = z0();
        omg[2 * F + oj] = z0();
      }
    }
  }
  const int s = sign ? d.mz - labs : labs;
  const int64_t o = reg ? (int64_t)s * d.mt + n : 0;
  const double a = n * d.kt, b = (sign ? -labs : labs) * d.kz;
  const bool zero_mode = labs == 0 && n == 0;
  const double* fl = flin + (int64_t)dmc * LINE_Q * 2 * LPS + 2 * ch;
  const int64_t fop = (int64_t)d.ndm * LINE_Q * 2 * LPS;
  auto IR = [&](int r) { return tab[(r * TAB_F + TAB_IR) * LPS + ch]; };
  auto V = [&](int c, int r) -> cd& { return vel[((wv * 3 + c) * RPL + r) * NLANE + lane]; };
  cd w[RPL + 2 * HW], rp[RPL];

  // 1. Ne = 2 N^i - N^{i-1} (kept in vel) and the pressure right-hand side
  //    -D(Ne), with the consistent Neumann rows at the walls
  {
    cd er[RPL], l[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int64_t oj = (int64_t)(j0 + r) * S + o;
      cd e3[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        e3[c] = csub(scl(N[c * F + oj], 2.0), Np[c * F + oj]);
        V(c, r) = e3[c];
      }
      const double ir = IR(r);
      er[r] = scl(cadd(e3[0], e3[1]), 0.5);
      cd lr = scl(er[r], ir);
      lr = fmac(lr, 0.5 * a * ir, csub(e3[0], e3[1]));
      l[r] = cadd(lr, imul(e3[2], b));
    }
    halo<LPS>(er, w, lane, ch);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const cd acc = cadd(d1_at<LPS>(tab, ch, r, w), l[r]);
      rp[r] = cd{-acc.x, -acc.y};
    }
    if (ch == 0 || ch == LPS - 1) {
      // V_r(2 u^i - u^{i-1}) at the wall, V_r = (L+ u+ + L- u-)/2, from the
      // 5 rows next to it (all in this lane)
      const int jw = ch ? M : 0;
      const double* R = rc + (int64_t)jw * RC_N;
      cd bc = z0();
#pragma unroll
      for (int jj = 0; jj <= HW; ++jj) {
        const int j = ch ? M - HW + jj : jj;
        const int k = j - jw + HW;
        const int64_t oj = (int64_t)j * S + o;
        const cd vp = csub(scl(u[oj], 2.0), up[oj]);
        const cd vm = csub(scl(u[F + oj], 2.0), up[F + oj]);
        const cd sum = cadd(vp, vm), dif = csub(vp, vm);
        cd tt = scl(sum, 0.5 * (R[RC_W2 + k] + R[RC_W1 + k] * R[RC_IR]));
        if (k == HW) {
          tt = fmac(tt, 0.5 * (-(a * a + 1.0) * R[RC_IR2] - b * b), sum);
          tt = fmac(tt, -a * R[RC_IR2], dif);
        }
        bc = cadd(bc, tt);
      }
      if (ch == 0) rp[0] = scl(csub(bc, er[0]), d.s0);
      else rp[RPL - 1] = zero_mode ? z0() : scl(csub(bc, er[RPL - 1]), d.sM);
    }
  }

  // 2. p* (P, LU)
  line_op_solve<LPS, true>(fl + OP_P * fop, rp, lane, ch);
  cd ps[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) ps[r] = rp[r];

  // 3. right-hand sides of the three Helmholtz problems, then u* (in vel)
  {
    const double c_dt = 1.0 / (2.0 * d.dt);
    halo<LPS>(ps, w, lane, ch);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int64_t oj = (int64_t)(j0 + r) * S + o;
      const double ir = IR(r);
      const cd d1 = d1_at<LPS>(tab, ch, r, w);
      const cd pi = ps[r];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cd ut = csub(scl(u[c * F + oj], 4.0), up[c * F + oj]);
        const cd e = V(c, r);
        cd h = cd{e.x - ut.x * c_dt, e.y - ut.y * c_dt};
        if (c == 0) h = cadd(h, nfmac(d1, a * ir, pi));
        if (c == 1) h = cadd(h, fmac(d1, a * ir, pi));
        if (c == 2) h = cadd(h, imul(pi, b));
        V(c, r) = h;
      }
    }
    if (ch == 0 || ch == LPS - 1) {
      const int r = ch ? RPL - 1 : 0;
      const double Re = ch ? d.Re_o : d.Re_i;
      V(0, r) = zero_mode ? cd{0.0, Re} : z0();
      V(1, r) = zero_mode ? cd{0.0, -Re} : z0();
      V(2, r) = z0();
    }
  }
#pragma unroll 1
  for (int c = 0; c < 3; ++c) {
    cd f[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) f[r] = V(c, r);
    line_op_solve<LPS, false>(fl + (OP_HP + c) * fop, f, lane, ch);
#pragma unroll
    for (int r = 0; r < RPL; ++r) V(c, r) = f[r];
  }

  // 4. phi: P phi = D(u*) (homogeneous Neumann rows)
  {
    cd ur[RPL], l[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const cd x0 = V(0, r), x1 = V(1, r), x2 = V(2, r);
      const double ir = IR(r);
      ur[r] = scl(cadd(x0, x1), 0.5);
      cd lr = scl(ur[r], ir);
      lr = fmac(lr, 0.5 * a * ir, csub(x0, x1));
      l[r] = cadd(lr, imul(x2, b));
    }
    halo<LPS>(ur, w, lane, ch);
#pragma unroll
    for (int r = 0; r < RPL; ++r) rp[r] = cadd(d1_at<LPS>(tab, ch, r, w), l[r]);
    if (ch == 0) rp[0] = z0();
    if (ch == LPS - 1) rp[RPL - 1] = z0();
  }
  line_op_solve<LPS, true>(fl + OP_P * fop, rp, lane, ch);

  // 5. correction u^{i+1} = u* - grad phi, p = p* + 3 phi / (2 dt)
  //    (mode (0,0): the correction removes u*_r, the exact solution of the
  //    correction equation for that mode)
  {
    const double c_p = 1.5 / d.dt;
    halo<LPS>(rp, w, lane, ch);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int64_t oj = (int64_t)(j0 + r) * S + o;
      const double ir = IR(r);
      const cd d1 = d1_at<LPS>(tab, ch, r, w);
      const cd ph = rp[r];
      const cd x0 = V(0, r), x1 = V(1, r), x2 = V(2, r);
      cd v0 = csub(x0, nfmac(d1, a * ir, ph));
      cd v1 = csub(x1, fmac(d1, a * ir, ph));
      const cd v2 = csub(x2, imul(ph, b));
      if (zero_mode) {
        v0 = scl(csub(x0, x1), 0.5);
        v1 = cd{-v0.x, -v0.y};
      }
      if (reg) {
        un[oj] = v0;
        un[F + oj] = v1;
        un[2 * F + oj] = v2;
        if (want_p) p[oj] = fmac(ps[r], c_p, ph);
      }
      if (FUSE) {
        V(0, r) = v0;
        V(1, r) = v1;
        V(2, r) = v2;
      }
    }
  }

  // 6. omega = curl u^{i+1} for the next step's nonlinear term
  if (FUSE) {
    cd xr[RPL], dp[RPL], dmn[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) xr[r] = V(0, r);
    halo<LPS>(xr, w, lane, ch);
#pragma unroll
    for (int r = 0; r < RPL; ++r) dp[r] = d1_at<LPS>(tab, ch, r, w);
#pragma unroll
    for (int r = 0; r < RPL; ++r) xr[r] = V(1, r);
    halo<LPS>(xr, w, lane, ch);
#pragma unroll
    for (int r = 0; r < RPL; ++r) dmn[r] = d1_at<LPS>(tab, ch, r, w);
#pragma unroll
    for (int r = 0; r < RPL; ++r) xr[r] = V(2, r);
    halo<LPS>(xr, w, lane, ch);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int64_t oj = (int64_t)(j0 + r) * S + o;
      const double ir = IR(r);
      const cd dz = d1_at<LPS>(tab, ch, r, w);
      const cd upv = V(0, r), umv = V(1, r), uzv = xr[r];
      // omega+ = i (a/r uz - D1 uz) - b u+ ;  omega- = i (a/r uz + D1 uz) + b u-
      const cd tp = {a * ir * uzv.x - dz.x, a * ir * uzv.y - dz.y};
      const cd tm = {a * ir * uzv.x + dz.x, a * ir * uzv.y + dz.y};
      const cd op = {-tp.y - b * upv.x, tp.x - b * upv.y};
      const cd om = {-tm.y + b * umv.x, tm.x + b * umv.y};
      // omega_z = -(i/2) [ (D1 + (1+a)/r) u+ - (D1 + (1-a)/r) u- ]
      const cd qz = {dp[r].x + (1.0 + a) * ir * upv.x - dmn[r].x - (1.0 - a) * ir * umv.x,
                     dp[r].y + (1.0 + a) * ir * upv.y - dmn[r].y - (1.0 - a) * ir * umv.y};
      if (reg) {
        omg[oj] = op;
        omg[F + oj] = om;
        omg[2 * F + oj] = cd{0.5 * qz.y, -0.5 * qz.x};
      }
    }
  }
}

// Transposed solves A^T x = rhs on the same line layout (the adjoint
// step's P and Helmholtz solves), A = S^-1 L U in the factor's row order
// (S: the Neumann row scale of P, identity for the Helmholtz operators):
//   U^T w = rhs   w_i = (rhs_i - sum_c U(i-c, i) w_{i-c}) / U(i, i)
//   L^T v = w     v_i = w_i - sum_q L(i+1+q, i) v_{i+1+q}
//   x = S v
// in the operator's processing order i.  The coefficients of row i come from
// the 4 rows before it (U^T) or after it (L^T) in that order, so each lane
// takes 4 rows of U coefficients from one neighbour and 4 rows of
// multipliers from the other by shuffles.  Operators op0 .. op0 + nop - 1 on
// fields rhs + k F -> x + k F (x may alias rhs: each lane reads its rows
// before it writes them).
template <int LPS, bool LU>
__device__ __forceinline__ void line_solve_t(const double* fl, cd (&f)[RPL], int lane, int ch) {
  double m[RPL][4], uc[RPL][4], ip[RPL];
  load_first<LPS>(fl, m);
  load_second<LPS>(fl, ip, uc);
  // neighbours' rows: the lane before (rows 4..7 of its slot) and after
  // (rows 0..3), zero past the ends of the line
  const int prev = (lane - 1) & (NLANE - 1), next = (lane + 1) & (NLANE - 1);
  double ua[HW][4], mb[HW][4];  // U rows feeding U^T, multiplier rows feeding L^T
#pragma unroll
  for (int i = 0; i < HW; ++i)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      // LU (ascending rows): U^T needs the rows before (lane - 1's rows 4..7),
      // L^T the rows after (lane + 1's rows 0..3); UL the other way round
      const double a = __shfl(uc[LU ? RPL - HW + i : i][c], LU ? prev : next, NLANE);
      const double b = __shfl(m[LU ? i : RPL - HW + i][c], LU ? next : prev, NLANE);
      ua[i][c] = (LU ? ch == 0 : ch == LPS - 1) ? 0.0 : a;
      mb[i][c] = (LU ? ch == LPS - 1 : ch == 0) ? 0.0 : b;
    }
  // coefficient of the c-th previous output, by row, for each recurrence
  double ca[RPL][4], cb[RPL][4];
#pragma unroll
  for (int r = 0; r < RPL; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      // U^T: row r's coefficient c is U(row i-1-c, entry c+1), i the
      // processing place of row r (rows r-1-c for LU, r+1+c for UL)
      const int ra = LU ? r - 1 - c : r + 1 + c;
      ca[r][c] = (ra >= 0 && ra < RPL) ? uc[ra][c] : ua[LU ? ra + HW : ra - RPL][c];
      // L^T: multiplier c of row i+1+c (rows r+1+c for LU, r-1-c for UL)
      const int rb = LU ? r + 1 + c : r - 1 - c;
      cb[r][c] = (rb >= 0 && rb < RPL) ? m[rb][c] : mb[LU ? rb - RPL : rb + HW][c];
    }
  line_solve<LPS, LU, true>(ca, ip, f, lane, ch);
  line_solve<LPS, !LU, false>(cb, ip, f, lane, ch);
}

template <int LPS>
__global__ __launch_bounds__(WAVES * NLANE) void k_solve_tl(const double* __restrict__ flin, Dims d, int op0, int nop,
                                                           const cd* rhs, cd* x, int ntile, int per) {
  constexpr int SPW = NLANE / LPS;
  const int lane = threadIdx.x % NLANE, wv = threadIdx.x / NLANE;
  const int seg = lane / LPS, ch = lane % LPS;
  const int xcd = blockIdx.x % 8, rr = blockIdx.x / 8;
  const int t = xcd * per + rr / 8, q = rr % 8;
  if (t >= ntile) return;
  const int sign = q & 1;
  const int dm = ((t * 4 + (q >> 1)) * WAVES + wv) * SPW + seg;
  const bool active = dm < d.ndm;
  if (__ballot(active) == 0) return;
  const int dmc = active ? dm : d.ndm - 1;
  const int labs = dmc / d.mt, n = dmc - labs * d.mt;
  const bool nyq = active && sign == 1 && labs == 0;
  const bool reg = active && !nyq;
  const int M = d.n_r - 1;
  const int64_t F = d.F, S = d.S;
  const int j0 = RPL * ch;
  const int s = sign ? d.mz - labs : labs;
  const int64_t o = reg ? (int64_t)s * d.mt + n : 0;
  const int64_t onyq = (int64_t)d.nyq * d.mt + n;
  const bool zero_mode = labs == 0 && n == 0;
  const double* fl = flin + (int64_t)dmc * LINE_Q * 2 * LPS + 2 * ch;
  const int64_t fop = (int64_t)d.ndm * LINE_Q * 2 * LPS;
#pragma unroll 1
  for (int k = 0; k < nop; ++k) {
    const int op = op0 + k;
    cd f[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) f[r] = rhs[k * F + (int64_t)(j0 + r) * S + o];
    if (op == OP_P) line_solve_t<LPS, true>(fl + op * fop, f, lane, ch);
    else line_solve_t<LPS, false>(fl + op * fop, f, lane, ch);
    if (op == OP_P) {
      // x = S v: the Neumann rows 0 and M (row M of mode (0,0) is Dirichlet)
      if (ch == 0) f[0] = scl(f[0], d.s0);
      if (ch == LPS - 1 && !zero_mode) f[RPL - 1] = scl(f[RPL - 1], d.sM);
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int64_t oj = k * F + (int64_t)(j0 + r) * S;
      if (reg) x[oj + o] = f[r];
      if (nyq) x[oj + onyq] = z0();
    }
  }
  (void)M;
}

// Adjoint of the predictor-corrector on the line layout: the chain of the
// adjoint step (tc_adjoint.hip) from the cotangent u_bar' of u^{i+1} and
// N_bar of N^i to the cotangents of u^i, u^{i-1}, N^{i-1} and the total
// cotangent of N(u^i), with every intermediate on chip:
//   phi_bar = -grad^H u_bar' (0 for mode (0,0))      r_phi = P^-T phi_bar
//   u*_bar = u_bar' + div^H(I r_phi)                 r_u = H^-T u*_bar
//   p_bar = grad^H(I r_u)                            r_p = P^-T p_bar
//   Ne_bar = I r_u - div^H(I r_p) - (W r_p)/2
//   u_bar = -(2/dt) I r_u + 2 V,  u_prev_bar = I r_u/(2dt) - V,
//   V = (L+^T W r_p, L-^T W r_p)/2 (zero past HW rows from the walls)
//   N_prev_bar = -Ne_bar,  N_tot = 2 Ne_bar + N_bar
// (I: interior rows, W: the wall rows of the consistent Neumann condition,
// not the outer row of mode (0,0)).  D1^T sums, for row k, the D1 weights
// of rows k-4 .. k+4 in column k, in that order; the per-row table holds
// those transposed weights.
template <int LPS>
__global__ __launch_bounds__(WAVES * NLANE) void k_pcl_adj(const double* __restrict__ rc,
                                                          const double* __restrict__ flin, Dims d,
                                                          const cd* __restrict__ ub, const cd* __restrict__ nin,
                                                          cd* __restrict__ out_u, cd* __restrict__ out_up,
                                                          cd* __restrict__ out_np, cd* __restrict__ ntot, int ntile,
                                                          int per) {
  constexpr int SPW = NLANE / LPS;
  __shared__ double tab[RPL * TAB_F * LPS];
  __shared__ cd vel[WAVES * 3 * RPL * NLANE];
  const int lane = threadIdx.x % NLANE, wv = threadIdx.x / NLANE;
  const int seg = lane / LPS, ch = lane % LPS;
  const int M = d.n_r - 1;
  // transposed D1 weights: entry m of row k multiplies row i = k + m - 4,
  // and is D1[i][k] (zero for rows past the walls)
  for (int i = threadIdx.x; i < RPL * TAB_F * LPS; i += blockDim.x) {
    const int k = i % LPS, rf = i / LPS, r = rf / TAB_F, f = rf % TAB_F;
    const int row = RPL * k + r;
    double v;
    if (f < NB9) {
      const int src = row + f - HW;
      v = (src >= 0 && src <= M) ? rc[(int64_t)src * RC_N + RC_W1 + (NB9 - 1 - f)] : 0.0;
    } else {
      v = rc[(int64_t)row * RC_N + RC_IR];
    }
    tab[i] = v;
  }
  __syncthreads();
  const int x = blockIdx.x % 8, rr = blockIdx.x / 8;
  const int t = x * per + rr / 8, q = rr % 8;
  if (t >= ntile) return;
  const int sign = q & 1;
  const int dm = ((t * 4 + (q >> 1)) * WAVES + wv) * SPW + seg;
  const bool active = dm < d.ndm;
  if (__ballot(active) == 0) return;
  const int dmc = active ? dm : d.ndm - 1;
  const int labs = dmc / d.mt, n = dmc - labs * d.mt;
  const bool nyq = active && sign == 1 && labs == 0;
  const bool reg = active && !nyq;
  const int64_t F = d.F, S = d.S;
  const int j0 = RPL * ch;
  if (nyq) {
    const int64_t on = (int64_t)d.nyq * d.mt + n;
#pragma unroll
    for (int r = 0; r < RPL; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t oj = c * F + (int64_t)(j0 + r) * S + on;
        out_u[oj] = z0();
        out_up[oj] = z0();
        out_np[oj] = z0();
        ntot[oj] = z0();
      }
  }
  const int s = sign ? d.mz - labs : labs;
  const int64_t o = reg ? (int64_t)s * d.mt + n : 0;
  const double a = n * d.kt, b = (sign ? -labs : labs) * d.kz;
  const bool zero_mode = labs == 0 && n == 0;
  const double* fl = flin + (int64_t)dmc * LINE_Q * 2 * LPS + 2 * ch;
  const int64_t fop = (int64_t)d.ndm * LINE_Q * 2 * LPS;
  auto IR = [&](int r) { return tab[(r * TAB_F + TAB_IR) * LPS + ch]; };
  auto V = [&](int c, int r) -> cd& { return vel[((wv * 3 + c) * RPL + r) * NLANE + lane]; };
  // interior rows of the line (wall rows: row 0 of lane 0, row 7 of the last lane)
  auto interior = [&](int r) { return !((ch == 0 && r == 0) || (ch == LPS - 1 && r == RPL - 1)); };
  cd w[RPL + 2 * HW], x1[RPL];
  const double c_dt = 1.0 / d.dt;

  // 1. phi_bar = -grad^H u_bar', grad^H v = D1^T (v+ + v-) - (a/r) v+ + (a/r) v- - i b v_z
  {
    cd sm[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int64_t oj = (int64_t)(j0 + r) * S + o;
#pragma unroll
      for (int c = 0; c < 3; ++c) V(c, r) = ub[c * F + oj];
      sm[r] = cadd(V(0, r), V(1, r));
    }
    halo<LPS>(sm, w, lane, ch);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      cd g = d1_at<LPS>(tab, ch, r, w);
      g = cadd(g, scl(csub(V(1, r), V(0, r)), a * IR(r)));
      g = csub(g, imul(V(2, r), b));
      x1[r] = zero_mode ? z0() : cd{-g.x, -g.y};
    }
  }
  // 2. r_phi = P^-T phi_bar
  line_solve_t<LPS, true>(fl + OP_P * fop, x1, lane, ch);
  if (ch == 0) x1[0] = scl(x1[0], d.s0);
  if (ch == LPS - 1 && !zero_mode) x1[RPL - 1] = scl(x1[RPL - 1], d.sM);
  // 3. u*_bar = u_bar' + div^H(I r_phi) (in vel; mode (0,0): the transpose
  //    of u^{i+1}+- = u*+- - u*_r maps (v+, v-) to ((v+ - v-)/2, (v- - v+)/2))
  {
    cd mr[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) mr[r] = interior(r) ? x1[r] : z0();
    halo<LPS>(mr, w, lane, ch);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const double ir = IR(r);
      const cd f = mr[r];
      const cd dt = scl(d1_at<LPS>(tab, ch, r, w), 0.5);
      cd vp = V(0, r), vm = V(1, r);
      if (zero_mode) {
        vp = scl(csub(V(0, r), V(1, r)), 0.5);
        vm = cd{-vp.x, -vp.y};
      }
      V(0, r) = cadd(vp, cadd(dt, scl(f, 0.5 * (1.0 + a) * ir)));
      V(1, r) = cadd(vm, cadd(dt, scl(f, 0.5 * (1.0 - a) * ir)));
      V(2, r) = csub(V(2, r), imul(f, b));
    }
  }
  // 4. r_u = H^-T u*_bar
#pragma unroll 1
  for (int c = 0; c < 3; ++c) {
    cd f[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) f[r] = V(c, r);
    line_solve_t<LPS, false>(fl + (OP_HP + c) * fop, f, lane, ch);
#pragma unroll
    for (int r = 0; r < RPL; ++r) V(c, r) = interior(r) ? f[r] : z0();  // I r_u
  }
  // 5. p_bar = grad^H(I r_u), then r_p = P^-T p_bar
  {
    cd sm[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) sm[r] = cadd(V(0, r), V(1, r));
    halo<LPS>(sm, w, lane, ch);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      cd g = d1_at<LPS>(tab, ch, r, w);
      g = cadd(g, scl(csub(V(1, r), V(0, r)), a * IR(r)));
      x1[r] = csub(g, imul(V(2, r), b));
    }
  }
  line_solve_t<LPS, true>(fl + OP_P * fop, x1, lane, ch);
  if (ch == 0) x1[0] = scl(x1[0], d.s0);
  if (ch == LPS - 1 && !zero_mode) x1[RPL - 1] = scl(x1[RPL - 1], d.sM);
  // 6. Ne_bar, the cotangents of u^i, u^{i-1}, N^{i-1} and N_tot
  {
    cd mr[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) mr[r] = interior(r) ? x1[r] : z0();
    halo<LPS>(mr, w, lane, ch);
    // wall terms: w_r at row 0 (lane 0) or row M (last lane; not for mode (0,0))
    const bool wl = (ch == 0) || (ch == LPS - 1 && !zero_mode);
    const int jw = ch == 0 ? 0 : M;
    const cd ww = ch == 0 ? x1[0] : x1[RPL - 1];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int j = j0 + r;
      const int64_t oj = (int64_t)j * S + o;
      const double ir = IR(r);
      const cd f = mr[r];
      const cd dt = scl(d1_at<LPS>(tab, ch, r, w), 0.5);
      cd ne[3] = {V(0, r), V(1, r), V(2, r)};  // I r_u
      cd ou[3], oup[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        ou[c] = scl(ne[c], -2.0 * c_dt);
        oup[c] = scl(ne[c], 0.5 * c_dt);
      }
      ne[0] = csub(ne[0], cadd(dt, scl(f, 0.5 * (1.0 + a) * ir)));
      ne[1] = csub(ne[1], cadd(dt, scl(f, 0.5 * (1.0 - a) * ir)));
      ne[2] = cadd(ne[2], imul(f, b));
      const int k = j - jw + HW;  // place of row j in the wall row's stencil
      if (wl && k >= 0 && k < NB9) {
        const cd wj = (j == jw) ? ww : z0();
        ne[0] = csub(ne[0], scl(wj, 0.5));
        ne[1] = csub(ne[1], scl(wj, 0.5));
        // L+-^T w = D2^T w + D1^T(w / r) - (a^2/r^2 + b^2 + (1 +- 2a)/r^2) w
        const double* Rw = rc + (int64_t)jw * RC_N;
        // column j of the wall row's stencils: weight k = j - jw + HW
        const cd t2 = scl(ww, Rw[RC_W2 + k]);
        const cd t1 = scl(scl(ww, Rw[RC_IR]), Rw[RC_W1 + k]);
        const cd base = cadd(t2, t1);
        const double ir2 = rc[(int64_t)j * RC_N + RC_IR2];
        const double dd = a * a * ir2 + b * b;
        const cd vp = scl(csub(base, scl(wj, dd + (1.0 + 2.0 * a) * ir2)), 0.5);
        const cd vm = scl(csub(base, scl(wj, dd + (1.0 - 2.0 * a) * ir2)), 0.5);
        ou[0] = cadd(ou[0], scl(vp, 2.0));
        ou[1] = cadd(ou[1], scl(vm, 2.0));
        oup[0] = csub(oup[0], vp);
        oup[1] = csub(oup[1], vm);
      }
      if (reg) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          out_u[c * F + oj] = ou[c];
          out_up[c * F + oj] = oup[c];
          out_np[c * F + oj] = cd{-ne[c].x, -ne[c].y};
          ntot[c * F + oj] = cadd(scl(ne[c], 2.0), nin[c * F + oj]);
        }
      }
    }
  }
}

// Lanes per slot where the line kernel runs: n_r = 8 LPS with LPS = 4, 8
// or 16.  Longer lines need 32 or 64 lanes per slot, whose loads touch as
// many cache lines per instruction; there the four-sweep kernels, which
// stream whole cache lines at HBM speed, are faster.
int line_lps(const Dims& d) {
  if (d.n_r % RPL != 0) return 0;
  const int lps = d.n_r / RPL;
  return (lps == 4 || lps == 8 || lps == 16) ? lps : 0;
}

template <int LPS>
static hipError_t launch_lps(tc_ctx* c, const cd* u, const cd* u_prev, const cd* N, const cd* N_prev, cd* u_next,
                             cd* p, int want_p, cd* omg) {
  const Dims& d = c->d;
  constexpr int SPW = NLANE / LPS;
  const int ntile = (d.ndm + 16 * SPW - 1) / (16 * SPW);
  const int per = (ntile + 7) / 8;
  const dim3 grid(64 * per), block(WAVES * NLANE);
  if (omg)
    hipLaunchKernelGGL((k_pcl<LPS, true>), grid, block, 0, c->stream, c->rc_dev, c->flin, d, u, u_prev, N, N_prev,
                       u_next, p, want_p, omg, ntile, per);
  else
    hipLaunchKernelGGL((k_pcl<LPS, false>), grid, block, 0, c->stream, c->rc_dev, c->flin, d, u, u_prev, N, N_prev,
                       u_next, p, want_p, omg, ntile, per);
  return hipGetLastError();
}

template <int LPS>
static hipError_t launch_solve_t_lps(tc_ctx* c, int op0, int nop, const cd* rhs, cd* x) {
  const Dims& d = c->d;
  constexpr int SPW = NLANE / LPS;
  const int ntile = (d.ndm + 16 * SPW - 1) / (16 * SPW);
  const int per = (ntile + 7) / 8;
  hipLaunchKernelGGL((k_solve_tl<LPS>), dim3(64 * per), dim3(WAVES * NLANE), 0, c->stream, c->flin, d, op0, nop, rhs,
                     x, ntile, per);
  return hipGetLastError();
}

hipError_t launch_solve_t_line(tc_ctx* c, int op0, int nop, const cd* rhs, cd* x) {
  switch (line_lps(c->d)) {
    case 4: return launch_solve_t_lps<4>(c, op0, nop, rhs, x);
    case 8: return launch_solve_t_lps<8>(c, op0, nop, rhs, x);
    case 16: return launch_solve_t_lps<16>(c, op0, nop, rhs, x);
    default: return hipErrorInvalidValue;
  }
}

template <int LPS>
static hipError_t launch_pc_adj_lps(tc_ctx* c, const cd* ub, const cd* nin, cd* out_u, cd* out_up, cd* out_np,
                                    cd* ntot) {
  const Dims& d = c->d;
  constexpr int SPW = NLANE / LPS;
  const int ntile = (d.ndm + 16 * SPW - 1) / (16 * SPW);
  const int per = (ntile + 7) / 8;
  hipLaunchKernelGGL((k_pcl_adj<LPS>), dim3(64 * per), dim3(WAVES * NLANE), 0, c->stream, c->rc_dev, c->flin, d, ub,
                     nin, out_u, out_up, out_np, ntot, ntile, per);
  return hipGetLastError();
}

hipError_t launch_pc_adj_line(tc_ctx* c, const cd* ub, const cd* nin, cd* out_u, cd* out_up, cd* out_np, cd* ntot) {
  switch (line_lps(c->d)) {
    case 4: return launch_pc_adj_lps<4>(c, ub, nin, out_u, out_up, out_np, ntot);
    case 8: return launch_pc_adj_lps<8>(c, ub, nin, out_u, out_up, out_np, ntot);
    case 16: return launch_pc_adj_lps<16>(c, ub, nin, out_u, out_up, out_np, ntot);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pc_line(tc_ctx* c, const cd* u, const cd* u_prev, const cd* N, const cd* N_prev, cd* u_next,
                          cd* p, int want_p, cd* omg) {
  switch (line_lps(c->d)) {
    case 4: return launch_lps<4>(c, u, u_prev, N, N_prev, u_next, p, want_p, omg);
    case 8: return launch_lps<8>(c, u, u_prev, N, N_prev, u_next, p, want_p, omg);
    case 16: return launch_lps<16>(c, u, u_prev, N, N_prev, u_next, p, want_p, omg);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tc
