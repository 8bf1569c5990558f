// Banded LU factorisation, banded solves and the fused predictor-corrector
// step (Sec. 3.2, steps 2-5 of the paper; factors once, substitutions per
// step as the paper's last paragraph of Sec. 3.2 prescribes).
//
// Work decomposition: one lane per distinct mode (|l|, n).  A lane serves
// both axial slots +l and -l, whose operators are identical (they depend on
// l^2 only), so every factor load is used twice.  Lanes of a wave hold
// consecutive n, so every load and store of a radial row is one contiguous
// run per slot in the [j][s][n] layout: no transposition is needed between
// the transform layout and the solves.
//
// Factor layout and row order: see tc_internal.h.  The pressure operator P
// is factored with rows taken in ascending order (LU), the three Helmholtz
// operators in descending order (UL).  A solve with P therefore ends on a
// descending sweep and a Helmholtz solve starts with one, so the
// back-substitution of p* and the first sweep for u* share one pass over
// the rows; likewise u*'s second sweep and phi's first sweep share the next
// ascending pass.  The whole step is four passes over the radial rows.
//
// No pivoting: the Neumann rows of P are rescaled to the size of the
// neighbouring Laplacian rows, and the factorisation reports any zero or
// non-finite pivot.
//
// On large grids the first sweeps (P's forward sweeps in k_pc1 and k_pc3,
// the Helmholtz operators' in k_pc2) rebuild their multipliers row by row
// from the operator rows instead of loading them: the elimination that
// k_factor runs, in the same order and without contraction, so the values
// are the stored ones bit for bit.  Only the second-sweep coefficients,
// which the elimination produces in the opposite row order, come from
// memory.
#include "tc_solve_dev.h"

namespace tc {

struct ModeLane {
  int dm, labs, n;
  int64_t o[2];  // plane offsets of slots +l and -l
  double a, b[2];
  bool zero_mode;
};

__device__ __forceinline__ bool make_lane(const Dims& d, ModeLane& L) {
  L.dm = blockIdx.x * blockDim.x + threadIdx.x;
  if (L.dm >= d.ndm) return false;
  L.labs = L.dm / d.mt;
  L.n = L.dm - L.labs * d.mt;
  const int s1 = L.labs;
  const int s2 = L.labs ? d.mz - L.labs : 0;
  L.o[0] = (int64_t)s1 * d.mt + L.n;
  L.o[1] = (int64_t)s2 * d.mt + L.n;
  L.a = L.n * d.kt;
  L.b[0] = L.labs * d.kz;
  L.b[1] = -L.labs * d.kz;
  L.zero_mode = (L.labs == 0 && L.n == 0);
  return true;
}

// ------------------------------------------------------------------ factor
__global__ void k_factor(const double* __restrict__ rc, double* __restrict__ fac, double* __restrict__ flin, Dims d,
                         int* bad) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= NOPS * d.ndm) return;
  const int op = gid / d.ndm, dm = gid - op * d.ndm;
  const int labs = dm / d.mt, n = dm - labs * d.mt;
  const double a = n * d.kt, b = labs * d.kz;
  const bool rev = (op != OP_P);
  const int M = d.n_r - 1;
  Elim E;
  E.reset();
  int flag = 0;
  for (int ip = 0; ip <= M; ++ip) {
    const int j = rev ? M - ip : ip;
    double nat[NB9], row[NB9], mult[4];
    operator_row(rc, d, op, j, a, b, nat);
    for (int c = 0; c < NB9; ++c) row[c] = rev ? nat[NB9 - 1 - c] : nat[c];
    E.next(row, ip, mult);
    double* F = const_cast<double*>(facp(fac, d, op, j)) + dm;
    for (int q = 0; q < 4; ++q) F[(int64_t)q * d.ndm] = mult[q];
    const double piv = row[HW];
    if (!(fabs(piv) > 0.0) || !isfinite(piv)) flag = 1;
    double sec[5];  // inverse pivot, second-sweep coefficients
    sec[0] = E.U[0][0];
    for (int c = 1; c <= 4; ++c) sec[c] = (ip + c <= M) ? row[HW + c] : 0.0;
    for (int c = 0; c <= 4; ++c) F[(int64_t)(4 + c) * d.ndm] = sec[c];
    if (flin) {
      // the same values in the line kernel's lane-contiguous layout
      const int lps = d.n_r / LINE_RPL, k = j / LINE_RPL, r = j % LINE_RPL;
      double* Lp = flin + ((int64_t)op * d.ndm + dm) * LINE_Q * 2 * lps + 2 * k;
      auto put = [&](int e, double x) { Lp[(int64_t)(e / 2) * 2 * lps + (e % 2)] = x; };
      for (int q = 0; q < 4; ++q) put(4 * r + q, mult[q]);
      for (int c = 0; c <= 4; ++c) put(4 * LINE_RPL + 5 * r + c, sec[c]);
    }
  }
  if (flag) atomicOr(bad, 1);
}

hipError_t launch_factor(tc_ctx* c, int* bad_dev) {
  const int total = NOPS * c->d.ndm;
  hipLaunchKernelGGL(k_factor, dim3((total + 63) / 64), dim3(64), 0, c->stream, c->rc_dev, c->fac, c->flin, c->d,
                     bad_dev);
  return hipGetLastError();
}

// Check of the unpivoted factors (the paper's DGBTRF pivots): for every
// operator and distinct mode, solve A x = A x0 with x0_j = 1 + sin(0.7 j)/2
// by the stored factors and take the componentwise backward error
// max_j |A x - b|_j / (|A| |x| + |b|)_j (Oettli-Prager).  A backward-stable
// elimination gives a few units of rounding; element growth without
// pivoting would show here.  tmp: n_r doubles per (op, mode) lane; worst:
// the largest error over all lanes, as the bits of a non-negative double.
__global__ void k_factor_check(const double* __restrict__ rc, const double* __restrict__ fac, Dims d,
                               double* __restrict__ tmp, unsigned long long* worst) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = NOPS * d.ndm;
  if (gid >= total) return;
  const int op = gid / d.ndm, dm = gid - op * d.ndm;
  const int labs = dm / d.mt, n = dm - labs * d.mt;
  const double a = n * d.kt, b = labs * d.kz;
  const bool rev = (op != OP_P);
  const int M = d.n_r - 1;
  auto x0 = [](int j) { return 1.0 + 0.5 * sin(0.7 * j); };
  auto T = [&](int ip) -> double& { return tmp[(int64_t)ip * total + gid]; };
  // b = A x0 and the forward sweep, in the factor's row order
  double w[4] = {0.0, 0.0, 0.0, 0.0};
  for (int ip = 0; ip <= M; ++ip) {
    const int j = rev ? M - ip : ip;
    double row[NB9];
    operator_row(rc, d, op, j, a, b, row);
    double bj = 0.0;
    for (int k = 0; k < NB9; ++k) {
      const int node = j + k - HW;
      if (node >= 0 && node <= M) bj = fma(row[k], x0(node), bj);
    }
    const double* F = facp(fac, d, op, j) + dm;
    double y = bj;
    for (int q = 0; q < 4; ++q) y -= F[(int64_t)q * d.ndm] * w[q];
    for (int q = 3; q >= 1; --q) w[q] = w[q - 1];
    w[0] = y;
    T(ip) = y;
  }
  // back-substitution
  for (int q = 0; q < 4; ++q) w[q] = 0.0;
  for (int ip = M; ip >= 0; --ip) {
    const int j = rev ? M - ip : ip;
    const double* F = facp(fac, d, op, j) + dm;
    double y = T(ip);
    for (int c = 1; c <= 4; ++c) y -= F[(int64_t)(4 + c) * d.ndm] * w[c - 1];
    y *= F[(int64_t)4 * d.ndm];
    for (int q = 3; q >= 1; --q) w[q] = w[q - 1];
    w[0] = y;
    T(ip) = y;
  }
  // residual, row by row in natural order (x_j is T(ip(j)))
  double err = 0.0;
  for (int j = 0; j <= M; ++j) {
    double row[NB9];
    operator_row(rc, d, op, j, a, b, row);
    double r = 0.0, den = 0.0, bj = 0.0;
    for (int k = 0; k < NB9; ++k) {
      const int node = j + k - HW;
      if (node < 0 || node > M) continue;
      const double xk = T(rev ? M - node : node);
      r = fma(row[k], xk, r);
      den = fma(fabs(row[k]), fabs(xk), den);
      bj = fma(row[k], x0(node), bj);
    }
    r -= bj;
    den += fabs(bj);
    if (den > 0.0) err = fmax(err, fabs(r) / den);
  }
  if (!(err <= 1.0)) err = 1.0;  // a non-finite residual counts as the worst
  atomicMax(worst, (unsigned long long)__double_as_longlong(err));
}

hipError_t launch_factor_check(tc_ctx* c, double* tmp, unsigned long long* worst_dev) {
  const int total = NOPS * c->d.ndm;
  hipLaunchKernelGGL(k_factor_check, dim3((total + 63) / 64), dim3(64), 0, c->stream, c->rc_dev, c->fac, c->d, tmp,
                     worst_dev);
  return hipGetLastError();
}

// ------------------------------------------------------------------ standalone solve
// One operator, every mode.  The first sweep writes its intermediate into x,
// the second sweep overwrites it with the solution (x may alias rhs).
__global__ __launch_bounds__(64) void k_solve(const double* __restrict__ rc, const double* __restrict__ fac, Dims d,
                                              int op, const cd* rhs, cd* x) {
  ModeLane L;
  if (!make_lane(d, L)) return;
  const int M = d.n_r - 1;
  const bool rev = (op != OP_P);
  cd w[4][2];
  for (int q = 0; q < 4; ++q) w[q][0] = w[q][1] = cz();
  for (int ip = 0; ip <= M; ++ip) {
    const int j = rev ? M - ip : ip;
    const double* F = facp(fac, d, op, j) + L.dm;
    double scale = 1.0;
    if (op == OP_P) scale = (j == 0) ? d.s0 : (j == M ? d.sM : 1.0);
    if (op == OP_P && j == M && L.zero_mode) scale = 1.0;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      cd y = cmuls(rhs[j * d.S + L.o[m]], scale);
#pragma unroll
      for (int q = 0; q < 4; ++q) y = cnfma(y, F[(int64_t)q * d.ndm], w[q][m]);
      for (int q = 3; q >= 1; --q) w[q][m] = w[q - 1][m];
      w[0][m] = y;
    }
    x[j * d.S + L.o[0]] = w[0][0];
    x[j * d.S + L.o[1]] = w[0][1];
  }
  for (int q = 0; q < 4; ++q) w[q][0] = w[q][1] = cz();
  for (int ip = M; ip >= 0; --ip) {
    const int j = rev ? M - ip : ip;
    const double* F = facp(fac, d, op, j) + L.dm;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      cd y = x[j * d.S + L.o[m]];
#pragma unroll
      for (int c = 1; c <= 4; ++c) y = cnfma(y, F[(int64_t)(4 + c) * d.ndm], w[c - 1][m]);
      y = cmuls(y, F[(int64_t)4 * d.ndm]);
      for (int q = 3; q >= 1; --q) w[q][m] = w[q - 1][m];
      w[0][m] = y;
    }
    x[j * d.S + L.o[0]] = w[0][0];
    x[j * d.S + L.o[1]] = w[0][1];
    // the empty axial slot is written as zero (by the |l| = 0 lanes)
    if (L.labs == 0) x[j * d.S + (int64_t)d.nyq * d.mt + L.n] = cz();
  }
}

hipError_t launch_solve(tc_ctx* c, int op, int transposed, const cd* rhs, cd* x) {
  if (transposed) return launch_solve_t(c, op, 1, rhs, x);
  const int blocks = (c->d.ndm + 63) / 64;
  hipLaunchKernelGGL(k_solve, dim3(blocks), dim3(64), 0, c->stream, c->rc_dev, c->fac, c->d, op, rhs, x);
  return hipGetLastError();
}

// ------------------------------------------------------------------ fused predictor-corrector
// Sweeps (rows j = 0..M):
//  1 ascending : Ne = 2 N^i - N^{i-1} (kept in N_prev); RHS of the pressure
//                Poisson problem; forward sweep of P                      -> y_p   (in p)
//  2 descending: p* by back-substitution; RHS of the 3 Helmholtz problems;
//                first (descending) sweep of H+, H-, H_z                 -> z     (in u_next), p* (in p)
//  3 ascending : u* by the second sweep; RHS of phi; forward sweep of P  -> u* (in u_next), y_phi (in N_prev[0])
//  4 descending: phi by back-substitution; correction and pressure update -> u^{i+1} (in u_next), p
//                (mode (0,0): the correction removes u*_r entirely, the exact
//                solution of eq. correction for that mode)
// Stencil terms lag the sweep by 4 rows (the D1 stencil spans +-4 rows);
// in the ascending sweeps D1 is applied in scatter form (each new row adds
// its contribution to the 9 rows it touches), so no input window is kept.
// want_p = 0 skips the pressure update (p then holds scratch).
//
#define TC_PC_ARGS                                                                                              \
  const double *__restrict__ rc, const double *__restrict__ fac, Dims d, const cd *__restrict__ u, const cd *up, \
      const cd *__restrict__ N, cd *Np, cd *un, cd *p, int want_p, cd *omg

#ifndef PC_CH
#define PC_CH 4
#endif
#ifndef TC_FUSE_CURL
#define TC_FUSE_CURL 1
#endif
// Each sweep runs in three phases (rows that only enter the lagging
// stencil window, rows that do both parts, rows that only leave it), so the
// middle phase has no row-range branches and all of a row's loads are issued
// together at the top of its iteration: a lane waits for memory once per row.
template <int CH>
__global__ __launch_bounds__(64) void k_pc1(TC_PC_ARGS) {
  Lane1 L;
  if (!make_lane1(d, L)) return;
  const int M = d.n_r - 1;
  const int64_t F = d.F, S = d.S;
  const double a = L.a;
  // Wall rows of the consistent Neumann condition: 2 V_r(u^i) - V_r(u^{i-1})
  // = V_r(2 u^i - u^{i-1}), V_r = (L+ u+ + L- u-)/2, accumulated while the
  // sweep passes the 5 rows next to each wall.
  cd bc0 = cz(), bcM = cz();
  cd acc[NB9], yw[4], ner0 = cz(), nerM = cz();
  for (int k = 0; k < NB9; ++k) acc[k] = cz();
  for (int q = 0; q < 4; ++q) yw[q] = cz();
  auto load_row = [&](int j, cd (&nv)[3], cd (&pv)[3]) {
    const int64_t o = j * S + L.o;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      nv[c] = N[c * F + o];
      pv[c] = Np[c * F + o];
    }
  };
  // multipliers of P's forward sweep: rebuilt row by row in ascending order
  // by the one-row kernels (large grids, where the sweep streams at HBM
  // speed and the arithmetic is free), loaded by the chunked ones (small
  // grids, where the sweep is a latency chain that the arithmetic lengthens)
  Elim EP;
  EP.reset();
  auto load_fac = [&](int i, double (&fl)[4]) {
    if constexpr (CH == 1) {
      EP.row_mult(rc, d, OP_P, i, i, a, L.b, fl);
    } else {
      const double* Fp = facp(fac, d, OP_P, i) + L.dm;
#pragma unroll
      for (int q = 0; q < 4; ++q) fl[q] = Fp[(int64_t)q * d.ndm];
    }
  };
  // row j enters: Ne = 2 N^i - N^{i-1} (kept in N_prev), wall terms, D1 scatter
  auto feed = [&](int j, const cd (&nv)[3], const cd (&pv)[3]) {
    const double ir = rc[(int64_t)j * RC_N + RC_IR];
    const int64_t o = j * S + L.o;
    if (j <= HW || j >= M - HW) {
      const cd vp = csub(cmuls(u[o], 2.0), up[o]);
      const cd vm = csub(cmuls(u[F + o], 2.0), up[F + o]);
      const cd sum = cadd(vp, vm), dif = csub(vp, vm);
#pragma unroll
      for (int wsel = 0; wsel < 2; ++wsel) {
        const int jw = wsel ? M : 0;
        const int k = j - jw + HW;
        if (k < 0 || k >= NB9) continue;
        const double* R = rc + (int64_t)jw * RC_N;
        cd t = cmuls(sum, 0.5 * (R[RC_W2 + k] + R[RC_W1 + k] * R[RC_IR]));
        if (k == HW) {
          t = cfma(t, 0.5 * (-(a * a + 1.0) * R[RC_IR2] - L.b * L.b), sum);
          t = cfma(t, -a * R[RC_IR2], dif);
        }
        if (wsel) bcM = cadd(bcM, t); else bc0 = cadd(bc0, t);
      }
    }
    const cd ep = csub(cmuls(nv[0], 2.0), pv[0]);
    const cd em = csub(cmuls(nv[1], 2.0), pv[1]);
    const cd ez = csub(cmuls(nv[2], 2.0), pv[2]);
    Np[o] = ep;
    Np[F + o] = em;
    Np[2 * F + o] = ez;
    const cd er = cmuls(cadd(ep, em), 0.5);
    if (j == 0) ner0 = er;
    if (j == M) nerM = er;
    // D1 scatter: row j feeds rows i = j-4..j+4 (slot k = i - j + 4)
#pragma unroll
    for (int k = 0; k < NB9; ++k) {
      const int i = j - HW + k;
      if (i >= 0 && i <= M) acc[k] = cfma(acc[k], rc[(int64_t)i * RC_N + RC_W1 + (NB9 - 1 - k)], er);
    }
    cd l = cmuls(er, ir);
    l = cfma(l, 0.5 * a * ir, csub(ep, em));
    l = cadd(l, cimul(ez, L.b));
    acc[HW] = cadd(acc[HW], l);
  };
  // row i leaves the window: forward sweep of P -> y_p (in p)
  auto solve = [&](int i, const double (&fl)[4]) {
    cd rhs;
    if (i == 0) rhs = cmuls(csub(bc0, ner0), d.s0);
    else if (i == M) rhs = L.zero_mode ? cz() : cmuls(csub(bcM, nerM), d.sM);
    else rhs = cd{-acc[0].x, -acc[0].y};
#pragma unroll
    for (int q = 0; q < 4; ++q) rhs = cnfma(rhs, fl[q], yw[q]);
    for (int q = 3; q >= 1; --q) yw[q] = yw[q - 1];
    yw[0] = rhs;
    p[i * S + L.o] = rhs;
  };
  auto shift = [&]() {
    for (int k = 0; k < NB9 - 1; ++k) acc[k] = acc[k + 1];
    acc[NB9 - 1] = cz();
  };
  for (int j = 0; j < HW; ++j) {
    cd nv[3], pv[3];
    load_row(j, nv, pv);
    feed(j, nv, pv);
    shift();
  }
  if constexpr (CH == 1) {
    for (int j = HW; j <= M; ++j) {
      cd nv[3], pv[3];
      double fl[4];
      load_row(j, nv, pv);
      load_fac(j - HW, fl);
      feed(j, nv, pv);
      solve(j - HW, fl);
      shift();
    }
  } else {
    int j = HW;
    for (; j + CH - 1 <= M; j += CH) {
      cd nv[CH][3], pv[CH][3];
      double fl[CH][4];
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        load_row(j + r, nv[r], pv[r]);
        load_fac(j + r - HW, fl[r]);
      }
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        feed(j + r, nv[r], pv[r]);
        solve(j + r - HW, fl[r]);
        shift();
      }
    }
    for (; j <= M; ++j) {
      cd nv[3], pv[3];
      double fl[4];
      load_row(j, nv, pv);
      load_fac(j - HW, fl);
      feed(j, nv, pv);
      solve(j - HW, fl);
      shift();
    }
  }
  for (int j = M + 1; j <= M + HW; ++j) {
    double fl[4];
    load_fac(j - HW, fl);
    solve(j - HW, fl);
    shift();
  }
}

template <int CH>
__global__ __launch_bounds__(64) void k_pc2(TC_PC_ARGS) {
  Lane1 L;
  if (!make_lane1(d, L)) return;
  const int M = d.n_r - 1;
  const int64_t F = d.F, S = d.S;
  const double a = L.a;
  const double c_dt = 1.0 / (2.0 * d.dt);
  cd pw[NB9], zw[3][4];
  for (int k = 0; k < NB9; ++k) pw[k] = cz();
  for (int o = 0; o < 3; ++o)
    for (int q = 0; q < 4; ++q) zw[o][q] = cz();
  auto load_back = [&](int jj, cd& y, double (&fu)[5]) {
    const double* Fp = facp(fac, d, OP_P, jj) + L.dm;
#pragma unroll
    for (int c = 0; c < 5; ++c) fu[c] = Fp[(int64_t)(4 + c) * d.ndm];
    y = p[jj * S + L.o];
  };
  // multipliers of the Helmholtz operators' first sweeps: rebuilt row by
  // row in descending order by the one-row kernels, loaded by the chunked
  // ones (as for P in k_pc1)
  Elim EH[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) EH[c].reset();
  auto load_h = [&](int i, cd (&ne)[3], cd (&uu)[3], cd (&uq)[3], double (&fh)[3][4]) {
    const int64_t o = i * S + L.o;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ne[c] = Np[c * F + o];
      uu[c] = u[c * F + o];
      uq[c] = up[c * F + o];
      if constexpr (CH == 1) {
        EH[c].row_mult(rc, d, OP_HP + c, i, M - i, a, L.b, fh[c]);
      } else {
        const double* Fh = facp(fac, d, OP_HP + c, i) + L.dm;
#pragma unroll
        for (int q = 0; q < 4; ++q) fh[c][q] = Fh[(int64_t)q * d.ndm];
      }
    }
  };
  // back-substitution of p* at row jj
  auto back = [&](int jj, cd y, const double (&fu)[5]) {
#pragma unroll
    for (int c = 1; c <= 4; ++c) y = cnfma(y, fu[c], pw[c]);
    y = cmuls(y, fu[0]);
    pw[0] = y;
    if (want_p) p[jj * S + L.o] = y;
  };
  // RHS of the Helmholtz problems at row i and their first (descending) sweep
  auto hrow = [&](int i, const cd (&ne)[3], const cd (&uu)[3], const cd (&uq)[3], const double (&fh)[3][4]) {
    const double* R = rc + (int64_t)i * RC_N;
    const double ir = R[RC_IR];
    cd rhs[3];
    if (i == 0 || i == M) {
      const double Re = (i == 0) ? d.Re_i : d.Re_o;
      rhs[0] = L.zero_mode ? cd{0.0, Re} : cz();
      rhs[1] = L.zero_mode ? cd{0.0, -Re} : cz();
      rhs[2] = cz();
    } else {
      cd d1 = cz();
#pragma unroll
      for (int k = 0; k < NB9; ++k) d1 = cfma(d1, R[RC_W1 + k], pw[k]);
      const cd pi = pw[HW];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cd ut = csub(cmuls(uu[c], 4.0), uq[c]);
        cd r = cd{ne[c].x - ut.x * c_dt, ne[c].y - ut.y * c_dt};
        if (c == 0) r = cadd(r, cnfma(d1, a * ir, pi));
        if (c == 1) r = cadd(r, cfma(d1, a * ir, pi));
        if (c == 2) r = cadd(r, cimul(pi, L.b));
        rhs[c] = r;
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cd z = rhs[c];
#pragma unroll
      for (int q = 0; q < 4; ++q) z = cnfma(z, fh[c][q], zw[c][q]);
      for (int q = 3; q >= 1; --q) zw[c][q] = zw[c][q - 1];
      zw[c][0] = z;
      un[c * F + i * S + L.o] = z;
    }
  };
  auto shift = [&]() {
    for (int k = NB9 - 1; k >= 1; --k) pw[k] = pw[k - 1];
  };
  for (int jj = M; jj > M - HW; --jj) {
    cd y;
    double fu[5];
    load_back(jj, y, fu);
    shift();
    back(jj, y, fu);
  }
  if constexpr (CH == 1) {
    for (int jj = M - HW; jj >= 0; --jj) {
      cd y, ne[3], uu[3], uq[3];
      double fu[5], fh[3][4];
      load_back(jj, y, fu);
      load_h(jj + HW, ne, uu, uq, fh);
      shift();
      back(jj, y, fu);
      hrow(jj + HW, ne, uu, uq, fh);
    }
  } else {
    int jj = M - HW;
    for (; jj - (CH - 1) >= 0; jj -= CH) {
      cd y[CH], ne[CH][3], uu[CH][3], uq[CH][3];
      double fu[CH][5], fh[CH][3][4];
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        load_back(jj - r, y[r], fu[r]);
        load_h(jj - r + HW, ne[r], uu[r], uq[r], fh[r]);
      }
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        shift();
        back(jj - r, y[r], fu[r]);
        hrow(jj - r + HW, ne[r], uu[r], uq[r], fh[r]);
      }
    }
    for (; jj >= 0; --jj) {
      cd y, ne[3], uu[3], uq[3];
      double fu[5], fh[3][4];
      load_back(jj, y, fu);
      load_h(jj + HW, ne, uu, uq, fh);
      shift();
      back(jj, y, fu);
      hrow(jj + HW, ne, uu, uq, fh);
    }
  }
  for (int jj = -1; jj >= -HW; --jj) {
    cd ne[3], uu[3], uq[3];
    double fh[3][4];
    load_h(jj + HW, ne, uu, uq, fh);
    shift();
    pw[0] = cz();
    hrow(jj + HW, ne, uu, uq, fh);
  }
}

template <int CH>
__global__ __launch_bounds__(64) void k_pc3(TC_PC_ARGS) {
  Lane1 L;
  if (!make_lane1(d, L)) return;
  const int M = d.n_r - 1;
  const int64_t F = d.F, S = d.S;
  const double a = L.a;
  cd xw[3][4], acc[NB9], yp[4];
  for (int c = 0; c < 3; ++c)
    for (int q = 0; q < 4; ++q) xw[c][q] = cz();
  for (int k = 0; k < NB9; ++k) acc[k] = cz();
  for (int q = 0; q < 4; ++q) yp[q] = cz();
  auto load_row = [&](int j, cd (&zv)[3], double (&fh)[3][5]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double* Fh = facp(fac, d, OP_HP + c, j) + L.dm;
#pragma unroll
      for (int q = 0; q < 5; ++q) fh[c][q] = Fh[(int64_t)(4 + q) * d.ndm];
      zv[c] = un[c * F + j * S + L.o];
    }
  };
  // multipliers of P's forward sweep: rebuilt row by row in ascending order
  // by the one-row kernels (large grids, where the sweep streams at HBM
  // speed and the arithmetic is free), loaded by the chunked ones (small
  // grids, where the sweep is a latency chain that the arithmetic lengthens)
  Elim EP;
  EP.reset();
  auto load_fac = [&](int i, double (&fl)[4]) {
    if constexpr (CH == 1) {
      EP.row_mult(rc, d, OP_P, i, i, a, L.b, fl);
    } else {
      const double* Fp = facp(fac, d, OP_P, i) + L.dm;
#pragma unroll
      for (int q = 0; q < 4; ++q) fl[q] = Fp[(int64_t)q * d.ndm];
    }
  };
  // row j: u* by the second Helmholtz sweep, then its divergence scattered
  auto feed = [&](int j, const cd (&zv)[3], const double (&fh)[3][5]) {
    const double ir = rc[(int64_t)j * RC_N + RC_IR];
    cd xs[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cd y = zv[c];
#pragma unroll
      for (int q = 1; q <= 4; ++q) y = cnfma(y, fh[c][q], xw[c][q - 1]);
      y = cmuls(y, fh[c][0]);
      for (int q = 3; q >= 1; --q) xw[c][q] = xw[c][q - 1];
      xw[c][0] = y;
      un[c * F + j * S + L.o] = y;
      xs[c] = y;
    }
    const cd ur = cmuls(cadd(xs[0], xs[1]), 0.5);
#pragma unroll
    for (int k = 0; k < NB9; ++k) {
      const int i = j - HW + k;
      if (i >= 0 && i <= M) acc[k] = cfma(acc[k], rc[(int64_t)i * RC_N + RC_W1 + (NB9 - 1 - k)], ur);
    }
    cd l = cmuls(ur, ir);
    l = cfma(l, 0.5 * a * ir, csub(xs[0], xs[1]));
    l = cadd(l, cimul(xs[2], L.b));
    acc[HW] = cadd(acc[HW], l);
  };
  // row i: forward sweep of P for phi -> y_phi (in N_prev[0])
  auto solve = [&](int i, const double (&fl)[4]) {
    cd rhs = (i != 0 && i != M) ? acc[0] : cz();
#pragma unroll
    for (int q = 0; q < 4; ++q) rhs = cnfma(rhs, fl[q], yp[q]);
    for (int q = 3; q >= 1; --q) yp[q] = yp[q - 1];
    yp[0] = rhs;
    Np[i * S + L.o] = rhs;
  };
  auto shift = [&]() {
    for (int k = 0; k < NB9 - 1; ++k) acc[k] = acc[k + 1];
    acc[NB9 - 1] = cz();
  };
  for (int j = 0; j < HW; ++j) {
    cd zv[3];
    double fh[3][5];
    load_row(j, zv, fh);
    feed(j, zv, fh);
    shift();
  }
  if constexpr (CH == 1) {
    for (int j = HW; j <= M; ++j) {
      cd zv[3];
      double fh[3][5], fl[4];
      load_row(j, zv, fh);
      load_fac(j - HW, fl);
      feed(j, zv, fh);
      solve(j - HW, fl);
      shift();
    }
  } else {
    int j = HW;
    for (; j + CH - 1 <= M; j += CH) {
      cd zv[CH][3];
      double fh[CH][3][5], fl[CH][4];
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        load_row(j + r, zv[r], fh[r]);
        load_fac(j + r - HW, fl[r]);
      }
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        feed(j + r, zv[r], fh[r]);
        solve(j + r - HW, fl[r]);
        shift();
      }
    }
    for (; j <= M; ++j) {
      cd zv[3];
      double fh[3][5], fl[4];
      load_row(j, zv, fh);
      load_fac(j - HW, fl);
      feed(j, zv, fh);
      solve(j - HW, fl);
      shift();
    }
  }
  for (int j = M + 1; j <= M + HW; ++j) {
    double fl[4];
    load_fac(j - HW, fl);
    solve(j - HW, fl);
    shift();
  }
}

template <int CH>
__global__ __launch_bounds__(64) void k_pc4(TC_PC_ARGS) {
  Lane1 L;
  if (!make_lane1(d, L)) return;
  const int M = d.n_r - 1;
  const int64_t F = d.F, S = d.S;
  const double a = L.a;
  const double c_p = 1.5 / d.dt;
  const bool nyq_lane = (L.dm < d.mt) && (threadIdx.x < 32);  // |l| = 0, +l half: clears the empty slot
  cd fw[NB9];
  for (int k = 0; k < NB9; ++k) fw[k] = cz();
  auto load_back = [&](int jj, cd& y, double (&fu)[5]) {
    const double* Fp = facp(fac, d, OP_P, jj) + L.dm;
#pragma unroll
    for (int c = 0; c < 5; ++c) fu[c] = Fp[(int64_t)(4 + c) * d.ndm];
    y = Np[jj * S + L.o];
  };
  auto load_corr = [&](int i, cd (&us)[3], cd& pv) {
    const int64_t o = i * S + L.o;
#pragma unroll
    for (int c = 0; c < 3; ++c) us[c] = un[c * F + o];
    pv = want_p ? p[o] : cz();
  };
  // back-substitution of phi at row jj
  auto back = [&](cd y, const double (&fu)[5]) {
#pragma unroll
    for (int c = 1; c <= 4; ++c) y = cnfma(y, fu[c], fw[c]);
    fw[0] = cmuls(y, fu[0]);
  };
  // Fused curl of the new velocity (large grids, omg != NULL): the rows of
  // u^{i+1} enter a 9-row window as they are finished (descending), and
  // omega = curl u^{i+1} of row c is formed once rows c-4..c+4 are known,
  // with the arithmetic of the standalone curl kernel; the next step's
  // nonlinear term then needs no separate curl pass over u.
  cd uw[TC_FUSE_CURL && CH == 1 ? NB9 : 1][3];
  if constexpr (TC_FUSE_CURL && CH == 1)
    for (int k = 0; k < NB9; ++k) uw[k][0] = uw[k][1] = uw[k][2] = cz();
  auto curl_push = [&](int i, const cd (&v)[3]) {
    if constexpr (TC_FUSE_CURL && CH == 1) {
      for (int k = NB9 - 1; k >= 1; --k) {
        uw[k][0] = uw[k - 1][0]; uw[k][1] = uw[k - 1][1]; uw[k][2] = uw[k - 1][2];
      }
      uw[0][0] = v[0]; uw[0][1] = v[1]; uw[0][2] = v[2];
      const int c = i + HW;  // uw[k] holds row c - HW + k
      if (c > M) return;
      const double* R = rc + (int64_t)c * RC_N;
      const double ir = R[RC_IR];
      cd dp = cz(), dmn = cz(), dz = cz();
#pragma unroll
      for (int k = 0; k < NB9; ++k) {
        const double w = R[RC_W1 + k];
        dp.x = fma(w, uw[k][0].x, dp.x); dp.y = fma(w, uw[k][0].y, dp.y);
        dmn.x = fma(w, uw[k][1].x, dmn.x); dmn.y = fma(w, uw[k][1].y, dmn.y);
        dz.x = fma(w, uw[k][2].x, dz.x); dz.y = fma(w, uw[k][2].y, dz.y);
      }
      const cd upv = uw[HW][0], umv = uw[HW][1], uzv = uw[HW][2];
      const double b = L.b;
      // omega+ = i (a/r uz - D1 uz) - b u+ ;  omega- = i (a/r uz + D1 uz) + b u-
      const cd tp = {a * ir * uzv.x - dz.x, a * ir * uzv.y - dz.y};
      const cd tm = {a * ir * uzv.x + dz.x, a * ir * uzv.y + dz.y};
      const cd op = {-tp.y - b * upv.x, tp.x - b * upv.y};
      const cd om = {-tm.y + b * umv.x, tm.x + b * umv.y};
      // omega_z = -(i/2) [ (D1 + (1+a)/r) u+ - (D1 + (1-a)/r) u- ]
      const cd q = {dp.x + (1.0 + a) * ir * upv.x - dmn.x - (1.0 - a) * ir * umv.x,
                    dp.y + (1.0 + a) * ir * upv.y - dmn.y - (1.0 - a) * ir * umv.y};
      const int64_t o = c * S + L.o;
      omg[o] = op;
      omg[F + o] = om;
      omg[2 * F + o] = cd{0.5 * q.y, -0.5 * q.x};
      if (nyq_lane) {
        const int64_t on = c * S + (int64_t)d.nyq * d.mt + (L.dm % d.mt);
        omg[on] = cz(); omg[F + on] = cz(); omg[2 * F + on] = cz();
      }
    }
  };
  const bool fuse = TC_FUSE_CURL && CH == 1 && omg != nullptr;
  // correction and pressure update at row i
  auto correct = [&](int i, const cd (&us)[3], cd pv) {
    const double* R = rc + (int64_t)i * RC_N;
    const double ir = R[RC_IR];
    cd d1 = cz();
#pragma unroll
    for (int k = 0; k < NB9; ++k) d1 = cfma(d1, R[RC_W1 + k], fw[k]);
    const cd ph = fw[HW];
    const int64_t o = i * S + L.o;
    cd v[3] = {csub(us[0], cnfma(d1, a * ir, ph)), csub(us[1], cfma(d1, a * ir, ph)), csub(us[2], cimul(ph, L.b))};
    if (L.zero_mode) {
      // mode (0,0): d_r phi = u*_r solves eq. correction exactly for this
      // mode, so the radial velocity is removed and u_theta, u_z are kept
      v[0] = cmuls(csub(us[0], us[1]), 0.5);
      v[1] = cd{-v[0].x, -v[0].y};
    }
    un[o] = v[0];
    un[F + o] = v[1];
    un[2 * F + o] = v[2];
    if (fuse) curl_push(i, v);
    if (want_p) p[o] = cfma(pv, c_p, ph);
    if (nyq_lane) {
      const int64_t on = i * S + (int64_t)d.nyq * d.mt + (L.dm % d.mt);
      un[on] = cz(); un[F + on] = cz(); un[2 * F + on] = cz();
      if (want_p) p[on] = cz();
    }
  };
  auto shift = [&]() {
    for (int k = NB9 - 1; k >= 1; --k) fw[k] = fw[k - 1];
  };
  for (int jj = M; jj > M - HW; --jj) {
    cd y;
    double fu[5];
    load_back(jj, y, fu);
    shift();
    back(y, fu);
  }
  if constexpr (CH == 1) {
    for (int jj = M - HW; jj >= 0; --jj) {
      cd y, us[3], pv;
      double fu[5];
      load_back(jj, y, fu);
      load_corr(jj + HW, us, pv);
      shift();
      back(y, fu);
      correct(jj + HW, us, pv);
    }
  } else {
    int jj = M - HW;
    for (; jj - (CH - 1) >= 0; jj -= CH) {
      cd y[CH], us[CH][3], pv[CH];
      double fu[CH][5];
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        load_back(jj - r, y[r], fu[r]);
        load_corr(jj - r + HW, us[r], pv[r]);
      }
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        shift();
        back(y[r], fu[r]);
        correct(jj - r + HW, us[r], pv[r]);
      }
    }
    for (; jj >= 0; --jj) {
      cd y, us[3], pv;
      double fu[5];
      load_back(jj, y, fu);
      load_corr(jj + HW, us, pv);
      shift();
      back(y, fu);
      correct(jj + HW, us, pv);
    }
  }
  for (int jj = -1; jj >= -HW; --jj) {
    cd us[3], pv;
    load_corr(jj + HW, us, pv);
    shift();
    fw[0] = cz();
    correct(jj + HW, us, pv);
  }
  if (fuse) {
    // the last HW rows of omega: rows below the inner wall count as zero
    const cd zero3[3] = {cz(), cz(), cz()};
    for (int i = -1; i >= -HW; --i) curl_push(i, zero3);
  }
}

// Transposed solve A^T x = rhs with A = S^-1 L U (S: the Neumann row scale of
// P, identity for the Helmholtz operators), in the factor's row order:
// U^T w = rhs forwards, then L^T v = w backwards, then x = S v.
// NOP operators at once (ops op0..op0+NOP-1, fields
// rhs + k F -> x + k F), one mode per lane (the Lane1 layout of the
// predictor-corrector below).  Rows are taken CH at a time: the loads of a
// chunk are all issued before its recurrence runs, so a sweep waits for
// memory once per chunk rather than once per row (small problems, where
// there are too few waves to hide the latency, are bound by exactly that).
template <int NOP, int CH>
__global__ __launch_bounds__(64) void k_solve_tn(const double* __restrict__ fac, Dims d, int op0, const cd* rhs, cd* x) {
  Lane1 L;
  if (!make_lane1(d, L)) return;
  const int M = d.n_r - 1;
  const int64_t F = d.F, S = d.S;
  // ops 1-3 (Helmholtz) are factored in descending row order, P ascending
  const bool rev = (op0 != OP_P);
  auto row_of = [&](int ip) { return rev ? M - ip : ip; };
  auto fw = [&](int op, int ip, int c) { return facp(fac, d, op, row_of(ip))[(int64_t)c * d.ndm + L.dm]; };
  cd w[NOP][4];
#pragma unroll
  for (int k = 0; k < NOP; ++k)
#pragma unroll
    for (int q = 0; q < 4; ++q) w[k][q] = cz();
  // U^T w = rhs, in processing order
  for (int ip0 = 0; ip0 <= M; ip0 += CH) {
    cd r[CH][NOP];
    double inv[CH][NOP], uc[CH][NOP][4];
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int ip = ip0 + t;
      if (ip > M) continue;
      const int j = row_of(ip);
#pragma unroll
      for (int k = 0; k < NOP; ++k) {
        r[t][k] = rhs[k * F + j * S + L.o];
        inv[t][k] = fw(op0 + k, ip, 4);
#pragma unroll
        for (int c = 1; c <= 4; ++c) uc[t][k][c - 1] = (ip - c >= 0) ? fw(op0 + k, ip - c, 4 + c) : 0.0;
      }
    }
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int ip = ip0 + t;
      if (ip > M) continue;
      const int j = row_of(ip);
#pragma unroll
      for (int k = 0; k < NOP; ++k) {
        cd y = r[t][k];
#pragma unroll
        for (int c = 1; c <= 4; ++c) y = cnfma(y, uc[t][k][c - 1], w[k][c - 1]);
        y = cmuls(y, inv[t][k]);
#pragma unroll
        for (int q = 3; q >= 1; --q) w[k][q] = w[k][q - 1];
        w[k][0] = y;
        x[k * F + j * S + L.o] = y;
      }
    }
  }
  // L^T v = w backwards, then x = S v (S: Neumann row scale of P); the
  // |l| = 0, +l lanes also write the empty axial slot as zero
  const bool nyq_lane = (L.dm < d.mt) && (threadIdx.x < 32);
  const int64_t onyq = (int64_t)d.nyq * d.mt + L.dm;
#pragma unroll
  for (int k = 0; k < NOP; ++k)
#pragma unroll
    for (int q = 0; q < 4; ++q) w[k][q] = cz();
  for (int ip0 = M; ip0 >= 0; ip0 -= CH) {
    cd r[CH][NOP];
    double mc[CH][NOP][4];
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int ip = ip0 - t;
      if (ip < 0) continue;
      const int j = row_of(ip);
#pragma unroll
      for (int k = 0; k < NOP; ++k) {
        r[t][k] = x[k * F + j * S + L.o];
#pragma unroll
        for (int q = 1; q <= 4; ++q) mc[t][k][q - 1] = (ip + q <= M) ? fw(op0 + k, ip + q, q - 1) : 0.0;
      }
    }
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int ip = ip0 - t;
      if (ip < 0) continue;
      const int j = row_of(ip);
      double scale = 1.0;
      if (op0 == OP_P && !(j == M && L.zero_mode)) scale = (j == 0) ? d.s0 : (j == M ? d.sM : 1.0);
#pragma unroll
      for (int k = 0; k < NOP; ++k) {
        cd y = r[t][k];
#pragma unroll
        for (int q = 1; q <= 4; ++q) y = cnfma(y, mc[t][k][q - 1], w[k][q - 1]);
#pragma unroll
        for (int q = 3; q >= 1; --q) w[k][q] = w[k][q - 1];
        w[k][0] = y;
        x[k * F + j * S + L.o] = cmuls(y, scale);
        if (nyq_lane) x[k * F + j * S + onyq] = cz();
      }
    }
  }
}

hipError_t launch_solve_t(tc_ctx* c, int op0, int nop, const cd* rhs, cd* x) {
  if (c->flin && (nop == 1 || (nop == 3 && op0 == OP_HP))) return launch_solve_t_line(c, op0, nop, rhs, x);
  const int blocks = (c->d.ndm + 31) / 32;
  if (nop == 1)
    hipLaunchKernelGGL((k_solve_tn<1, 8>), dim3(blocks), dim3(64), 0, c->stream, c->fac, c->d, op0, rhs, x);
  else if (nop == 3 && op0 == OP_HP)
    hipLaunchKernelGGL((k_solve_tn<3, 4>), dim3(blocks), dim3(64), 0, c->stream, c->fac, c->d, op0, rhs, x);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Few waves (fewer than 2 per SIMD): too few to hide memory latency, so
// each lane loads PC_CH rows before working through them; otherwise one
// row at a time, which keeps the register count (and the occupancy that
// saturates HBM on large grids) down.
static bool pc_chunked(const tc_ctx* c) { return (c->d.ndm + 31) / 32 < 2 * 4 * 256; }

// (only the rotational form transforms the curl; the line kernel forms it
// on every grid it takes)
bool pc_fuses_curl(const tc_ctx* c) {
  return TC_FUSE_CURL && c->d.form == TC_ROTATIONAL && (c->flin || !pc_chunked(c));
}

hipError_t launch_pc(tc_ctx* c, const cd* u, const cd* u_prev, const cd* N, cd* N_prev, cd* u_next, cd* p,
                     int want_p, cd* omega_out) {
  cd* omg = pc_fuses_curl(c) ? omega_out : nullptr;
  if (c->flin) return launch_pc_line(c, u, u_prev, N, N_prev, u_next, p, want_p, omg);
  const int blocks = (c->d.ndm + 31) / 32;
  const bool chunked = pc_chunked(c);
  using K = void (*)(TC_PC_ARGS);
  const K ks[2][4] = {{k_pc1<1>, k_pc2<1>, k_pc3<1>, k_pc4<1>},
                      {k_pc1<PC_CH>, k_pc2<PC_CH>, k_pc3<PC_CH>, k_pc4<PC_CH>}};
  for (const K k : ks[chunked ? 1 : 0]) {
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64), 0, c->stream, c->rc_dev, c->fac, c->d, u, u_prev, N, N_prev,
                       u_next, p, want_p, omg);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace tc
