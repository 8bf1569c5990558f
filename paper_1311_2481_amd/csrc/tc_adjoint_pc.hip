// The predictor-corrector part of the adjoint step (tc_adjoint.hip) in four
// sweeps over the radial rows, for grids the line kernels do not take.  The
// chain, from the cotangent u_bar' of u^{i+1} and N_bar of N^i:
//   phi_bar = -grad^H u_bar' (0 for mode (0,0))      r_phi = P^-T phi_bar
//   u*_bar = u_bar' + div^H(I r_phi)                 r_u = H^-T u*_bar
//   p_bar = grad^H(I r_u)                            r_p = P^-T p_bar
//   Ne_bar = I r_u - div^H(I r_p) - (W r_p)/2
//   u_bar = -(2/dt) I r_u + 2 V,  u_prev_bar = I r_u/(2dt) - V,
//   V = (L+^T W r_p, L-^T W r_p)/2 (zero past HW rows from the walls)
//   N_prev_bar = -Ne_bar,  N_tot = 2 Ne_bar + N_bar
// (I: interior rows, W: the wall rows of the consistent Neumann condition,
// not the outer row of mode (0,0)).  A transposed solve A^T x = f with
// A = S^-1 L U takes two sweeps, U^T in the factor's row order and L^T
// against it, then x = S v; P's factor order is ascending and the
// Helmholtz operators' descending, so the chain alternates like the forward
// step's:
//   1 ascending : phi_bar (D1^T in scatter form), U_P^T sweep     -> w (wA)
//   2 descending: L_P^T -> r_phi; u*_bar; U_H^T sweeps of H+, H-, H_z -> (wH)
//   3 ascending : L_H^T -> r_u; u_bar, u_prev_bar; p_bar; U_P^T     -> (wA)
//   4 descending: L_P^T -> r_p; Ne_bar, the wall terms, N_prev_bar, N_tot
// (sweep 4 takes I r_u back from u_prev_bar = I r_u/(2dt), which sweep 3
// writes for every row before sweep 4 adds the wall terms).  The U^T sweeps
// run in the factor's own order.  Those of P (sweeps 1 and 3) rebuild their
// coefficients with the elimination of k_factor (bit for bit the stored
// ones); sweep 2 reads the stored U coefficients of the three Helmholtz
// operators, since three eliminations in one sweep cost more time than the
// reads.  The L^T sweeps read the stored multipliers.  D1^T(f) of row k
// sums D1[i][k] f_i over the rows i = k-4 .. k+4: each row adds its own
// stencil weights times f to the 9 rows it touches as it enters, and a
// row's sum is complete 4 rows later.
// Lanes as in the forward sweeps: one distinct mode per lane, its +l and -l
// slots in the two halves of a wave.
#include "tc_solve_dev.h"

namespace tc {

#define TC_PA_ARGS                                                                                            \
  const double *__restrict__ rc, const double *__restrict__ fac, Dims d, const cd *__restrict__ ub,          \
      const cd *__restrict__ nin, cd *__restrict__ out_u, cd *__restrict__ out_up, cd *__restrict__ out_np, \
      cd *__restrict__ ntot, cd *__restrict__ wA, cd *__restrict__ wH

namespace {

// scale of row j in x = S v for P (the Neumann rows; row M of mode (0,0) is Dirichlet)
__device__ __forceinline__ double s_of(const Dims& d, int j, bool zero_mode) {
  const int M = d.n_r - 1;
  if (j == 0) return d.s0;
  if (j == M && !zero_mode) return d.sM;
  return 1.0;
}

// one U^T step at processing place ip of operator op (row j): before the
// running elimination takes the row, U[c-1][c] is the entry U(ip - c, ip)
// of the c-th previous row; after it, U[0][0] is the row's inverse pivot
__device__ __forceinline__ cd ut_step(const double* rc, const Dims& d, Elim& E, int op, int j, int ip, double a,
                                      double b, cd f, cd (&w)[4]) {
  double cu[4], mult[4];
#pragma unroll
  for (int c = 1; c <= 4; ++c) cu[c - 1] = E.U[c - 1][c];
  E.row_mult(rc, d, op, j, ip, a, b, mult);
  cd y = f;
#pragma unroll
  for (int c = 1; c <= 4; ++c) y = cnfma(y, cu[c - 1], w[c - 1]);
  y = cmuls(y, E.U[0][0]);
#pragma unroll
  for (int q = 3; q >= 1; --q) w[q] = w[q - 1];
  w[0] = y;
  return y;
}

// one L^T step: v = f - sum_q m(q-th next row in processing order, q) v_next;
// mr[q] holds the multipliers of the row q+1 places before in this sweep
__device__ __forceinline__ cd lt_step(const double (&mr)[4][4], cd f, cd (&v)[4]) {
  cd y = f;
#pragma unroll
  for (int q = 0; q < 4; ++q) y = cnfma(y, mr[q][q], v[q]);
#pragma unroll
  for (int q = 3; q >= 1; --q) v[q] = v[q - 1];
  v[0] = y;
  return y;
}

// one U^T step from the stored factors: fu = (inverse pivot, U(ip, ip+1..ip+4))
// of this row, win[c-1][e-1] = U(ip-c, ip-c+e) of the row c places before
__device__ __forceinline__ cd ut_step_ld(const double (&fu)[5], double (&win)[4][4], cd f, cd (&w)[4]) {
  cd y = f;
#pragma unroll
  for (int c = 1; c <= 4; ++c) y = cnfma(y, win[c - 1][c - 1], w[c - 1]);
  y = cmuls(y, fu[0]);
#pragma unroll
  for (int q = 3; q >= 1; --q) {
    w[q] = w[q - 1];
#pragma unroll
    for (int e = 0; e < 4; ++e) win[q][e] = win[q - 1][e];
  }
  w[0] = y;
#pragma unroll
  for (int e = 0; e < 4; ++e) win[0][e] = fu[1 + e];
  return y;
}

__device__ __forceinline__ void push_mult(const double* fac, const Dims& d, int op, int j, int dm, double (&mr)[4][4]) {
#pragma unroll
  for (int q = 3; q >= 1; --q)
#pragma unroll
    for (int c = 0; c < 4; ++c) mr[q][c] = mr[q - 1][c];
  const double* Fp = facp(fac, d, op, j) + dm;
#pragma unroll
  for (int c = 0; c < 4; ++c) mr[0][c] = Fp[(int64_t)c * d.ndm];
}

// D1^T scatter of row j's value v into the window acc[k] = row j - 4 + k
__device__ __forceinline__ void scatter(const double* rc, const Dims& d, int j, cd v, cd (&acc)[NB9]) {
  const int M = d.n_r - 1;
  const double* R = rc + (int64_t)j * RC_N;
#pragma unroll
  for (int m = 0; m < NB9; ++m) {
    const int i = j - HW + m;
    if (i >= 0 && i <= M) acc[m] = cfma(acc[m], R[RC_W1 + m], v);
  }
}

}  // namespace

// 1. ascending: phi_bar and the U^T sweep of P -> wA
__global__ __launch_bounds__(64) void k_pa1(TC_PA_ARGS) {
  Lane1 L;
  if (!make_lane1(d, L)) return;
  const int M = d.n_r - 1;
  const int64_t F = d.F, S = d.S;
  const double a = L.a, b = L.b;
  Elim EP;
  EP.reset();
  cd acc[NB9], t1[HW + 1], t2[HW + 1], w[4];
  for (int k = 0; k < NB9; ++k) acc[k] = cz();
  for (int k = 0; k <= HW; ++k) t1[k] = t2[k] = cz();
  for (int q = 0; q < 4; ++q) w[q] = cz();
  // row i = j - 4 is complete: phi_bar, then U^T
  auto finish = [&](int i) {
    cd g = cadd(acc[0], t1[HW]);
    g = csub(g, t2[HW]);
    const cd pb = L.zero_mode ? cz() : cd{-g.x, -g.y};
    wA[i * S + L.o] = ut_step(rc, d, EP, OP_P, i, i, a, b, pb, w);
  };
  auto shift = [&]() {
    for (int k = 0; k < NB9 - 1; ++k) acc[k] = acc[k + 1];
    acc[NB9 - 1] = cz();
  };
  for (int j = 0; j <= M + HW; ++j) {
    // t1[k], t2[k]: local terms of row j - k
    for (int k = HW; k >= 1; --k) {
      t1[k] = t1[k - 1];
      t2[k] = t2[k - 1];
    }
    if (j <= M) {
      const int64_t o = j * S + L.o;
      const cd u0 = ub[o], u1 = ub[F + o], u2 = ub[2 * F + o];
      scatter(rc, d, j, cadd(u0, u1), acc);
      t1[0] = cmuls(csub(u1, u0), a * rc[(int64_t)j * RC_N + RC_IR]);
      t2[0] = cimul(u2, b);
    } else {
      t1[0] = t2[0] = cz();
    }
    if (j >= HW) finish(j - HW);
    shift();
  }
}

// 2. descending: L^T of P -> r_phi; u*_bar; the U^T sweeps of H+, H-, H_z -> wH
__global__ __launch_bounds__(64) void k_pa2(TC_PA_ARGS) {
  Lane1 L;
  if (!make_lane1(d, L)) return;
  const int M = d.n_r - 1;
  const int64_t F = d.F, S = d.S;
  const double a = L.a, b = L.b;
  double mr[4][4];
  for (int q = 0; q < 4; ++q)
    for (int c = 0; c < 4; ++c) mr[q][c] = 0.0;
  // U entries of the last 4 rows of each Helmholtz operator (loaded: at 3
  // operators, rebuilding the elimination in the sweep costs more time
  // than reading the coefficients)
  double win[3][4][4];
  for (int c = 0; c < 3; ++c)
    for (int q = 0; q < 4; ++q)
      for (int e = 0; e < 4; ++e) win[c][q][e] = 0.0;
  cd v[4], acc[NB9], fr[HW + 1], wh[3][4];
  for (int q = 0; q < 4; ++q) v[q] = cz();
  for (int k = 0; k < NB9; ++k) acc[k] = cz();
  for (int k = 0; k <= HW; ++k) fr[k] = cz();
  for (int c = 0; c < 3; ++c)
    for (int q = 0; q < 4; ++q) wh[c][q] = cz();
  // row r = i + 4 is complete (acc[NB9-1], fr[HW]): u*_bar and U^T of H
  auto finish = [&](int r) {
    const int64_t o = r * S + L.o;
    const double ir = rc[(int64_t)r * RC_N + RC_IR];
    const cd f = fr[HW];
    const cd dt = cmuls(acc[NB9 - 1], 0.5);
    cd vp = ub[o], vm = ub[F + o];
    if (L.zero_mode) {
      vp = cmuls(csub(ub[o], ub[F + o]), 0.5);
      vm = cd{-vp.x, -vp.y};
    }
    cd us[3];
    us[0] = cadd(vp, cadd(dt, cmuls(f, 0.5 * (1.0 + a) * ir)));
    us[1] = cadd(vm, cadd(dt, cmuls(f, 0.5 * (1.0 - a) * ir)));
    us[2] = csub(ub[2 * F + o], cimul(f, b));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double* Fh = facp(fac, d, OP_HP + c, r) + L.dm;
      double fu[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) fu[q] = Fh[(int64_t)(4 + q) * d.ndm];
      wH[c * F + o] = ut_step_ld(fu, win[c], us[c], wh[c]);
    }
  };
  auto shift = [&]() {
    for (int k = NB9 - 1; k >= 1; --k) acc[k] = acc[k - 1];
    acc[0] = cz();
    for (int k = HW; k >= 1; --k) fr[k] = fr[k - 1];
    fr[0] = cz();
  };
  for (int i = M; i >= -HW; --i) {
    if (i >= 0) {
      const cd y = lt_step(mr, wA[i * S + L.o], v);
      push_mult(fac, d, OP_P, i, L.dm, mr);
      const cd rphi = cmuls(y, s_of(d, i, L.zero_mode));
      const cd m = (i == 0 || i == M) ? cz() : rphi;  // I r_phi
      scatter(rc, d, i, m, acc);
      fr[0] = m;
    }
    if (i + HW <= M) finish(i + HW);
    shift();
  }
}

// 3. ascending: L^T of H+, H-, H_z -> r_u; u_bar, u_prev_bar; p_bar; the
//    U^T sweep of P -> wA
__global__ __launch_bounds__(64) void k_pa3(TC_PA_ARGS) {
  Lane1 L;
  if (!make_lane1(d, L)) return;
  const int M = d.n_r - 1;
  const int64_t F = d.F, S = d.S;
  const double a = L.a, b = L.b;
  const bool nyq_lane = (L.dm < d.mt) && (threadIdx.x < 32);
  const int64_t onyq = (int64_t)d.nyq * d.mt + (L.dm % d.mt);
  double mr[3][4][4];
  for (int c = 0; c < 3; ++c)
    for (int q = 0; q < 4; ++q)
      for (int e = 0; e < 4; ++e) mr[c][q][e] = 0.0;
  Elim EP;
  EP.reset();
  cd v[3][4], acc[NB9], t1[HW + 1], t2[HW + 1], w[4];
  for (int c = 0; c < 3; ++c)
    for (int q = 0; q < 4; ++q) v[c][q] = cz();
  for (int k = 0; k < NB9; ++k) acc[k] = cz();
  for (int k = 0; k <= HW; ++k) t1[k] = t2[k] = cz();
  for (int q = 0; q < 4; ++q) w[q] = cz();
  const double c2 = -2.0 / d.dt, ch = 0.5 / d.dt;
  auto finish = [&](int i) {
    cd g = cadd(acc[0], t1[HW]);
    g = csub(g, t2[HW]);
    wA[i * S + L.o] = ut_step(rc, d, EP, OP_P, i, i, a, b, g, w);
  };
  auto shift = [&]() {
    for (int k = 0; k < NB9 - 1; ++k) acc[k] = acc[k + 1];
    acc[NB9 - 1] = cz();
  };
  for (int j = 0; j <= M + HW; ++j) {
    for (int k = HW; k >= 1; --k) {
      t1[k] = t1[k - 1];
      t2[k] = t2[k - 1];
    }
    if (j <= M) {
      const int64_t o = j * S + L.o;
      cd m[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cd y = lt_step(mr[c], wH[c * F + o], v[c]);
        push_mult(fac, d, OP_HP + c, j, L.dm, mr[c]);
        m[c] = (j == 0 || j == M) ? cz() : y;  // I r_u
        out_u[c * F + o] = cmuls(m[c], c2);
        out_up[c * F + o] = cmuls(m[c], ch);
        if (nyq_lane) {
          const int64_t on = c * F + j * S + onyq;
          out_u[on] = out_up[on] = cz();
        }
      }
      scatter(rc, d, j, cadd(m[0], m[1]), acc);
      t1[0] = cmuls(csub(m[1], m[0]), a * rc[(int64_t)j * RC_N + RC_IR]);
      t2[0] = cimul(m[2], b);
    } else {
      t1[0] = t2[0] = cz();
    }
    if (j >= HW) finish(j - HW);
    shift();
  }
}

// 4. descending: L^T of P -> r_p; Ne_bar, the wall terms on u_bar and
//    u_prev_bar, N_prev_bar, N_tot
__global__ __launch_bounds__(64) void k_pa4(TC_PA_ARGS) {
  Lane1 L;
  if (!make_lane1(d, L)) return;
  const int M = d.n_r - 1;
  const int64_t F = d.F, S = d.S;
  const double a = L.a, b = L.b;
  const bool nyq_lane = (L.dm < d.mt) && (threadIdx.x < 32);
  const int64_t onyq = (int64_t)d.nyq * d.mt + (L.dm % d.mt);
  double mr[4][4];
  for (int q = 0; q < 4; ++q)
    for (int c = 0; c < 4; ++c) mr[q][c] = 0.0;
  cd v[4], acc[NB9], fr[HW + 1];
  for (int q = 0; q < 4; ++q) v[q] = cz();
  for (int k = 0; k < NB9; ++k) acc[k] = cz();
  for (int k = 0; k <= HW; ++k) fr[k] = cz();
  cd wr0 = cz(), wrM = cz();  // r_p at the wall rows that carry the Neumann condition
  auto finish = [&](int r) {
    const int64_t o = r * S + L.o;
    const double* R = rc + (int64_t)r * RC_N;
    const double ir = R[RC_IR];
    const cd f = fr[HW];
    const cd dt = cmuls(acc[NB9 - 1], 0.5);
    cd ne[3];
    // I r_u from u_prev_bar = I r_u / (2 dt), as sweep 3 wrote it (before
    // the wall terms below are added)
#pragma unroll
    for (int c = 0; c < 3; ++c) ne[c] = cmuls(out_up[c * F + o], 2.0 * d.dt);
    ne[0] = csub(ne[0], cadd(dt, cmuls(f, 0.5 * (1.0 + a) * ir)));
    ne[1] = csub(ne[1], cadd(dt, cmuls(f, 0.5 * (1.0 - a) * ir)));
    ne[2] = cadd(ne[2], cimul(f, b));
    if (r <= HW || r >= M - HW) {
      const cd w = (r == 0) ? wr0 : (r == M ? wrM : cz());
      ne[0] = csub(ne[0], cmuls(w, 0.5));
      ne[1] = csub(ne[1], cmuls(w, 0.5));
      // L+-^T w = D2^T w + D1^T(w / r) - (a^2/r^2 + b^2 + (1 +- 2a)/r^2) w,
      // w nonzero at the wall rows only
      cd t2 = cz(), t1 = cz();
#pragma unroll
      for (int wsel = 0; wsel < 2; ++wsel) {
        const int jw = wsel ? M : 0;
        const int k = r - jw + HW;
        if (k < 0 || k >= NB9) continue;
        const double* Rw = rc + (int64_t)jw * RC_N;
        const cd wv = wsel ? wrM : wr0;
        t2 = cfma(t2, Rw[RC_W2 + k], wv);
        t1 = cfma(t1, Rw[RC_W1 + k], cmuls(wv, Rw[RC_IR]));
      }
      const cd base = cadd(t2, t1);
      const double ir2 = R[RC_IR2];
      const double dd = a * a * ir2 + b * b;
      const cd vp = cmuls(csub(base, cmuls(w, dd + (1.0 + 2.0 * a) * ir2)), 0.5);
      const cd vm = cmuls(csub(base, cmuls(w, dd + (1.0 - 2.0 * a) * ir2)), 0.5);
      out_u[o] = cadd(out_u[o], cmuls(vp, 2.0));
      out_u[F + o] = cadd(out_u[F + o], cmuls(vm, 2.0));
      out_up[o] = csub(out_up[o], vp);
      out_up[F + o] = csub(out_up[F + o], vm);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      out_np[c * F + o] = cd{-ne[c].x, -ne[c].y};
      ntot[c * F + o] = cadd(cmuls(ne[c], 2.0), nin[c * F + o]);
      if (nyq_lane) {
        const int64_t on = c * F + r * S + onyq;
        out_np[on] = ntot[on] = cz();
      }
    }
  };
  auto shift = [&]() {
    for (int k = NB9 - 1; k >= 1; --k) acc[k] = acc[k - 1];
    acc[0] = cz();
    for (int k = HW; k >= 1; --k) fr[k] = fr[k - 1];
    fr[0] = cz();
  };
  for (int i = M; i >= -HW; --i) {
    if (i >= 0) {
      const cd y = lt_step(mr, wA[i * S + L.o], v);
      push_mult(fac, d, OP_P, i, L.dm, mr);
      const cd rp = cmuls(y, s_of(d, i, L.zero_mode));
      if (i == 0) wr0 = rp;
      if (i == M && !L.zero_mode) wrM = rp;
      const cd m = (i == 0 || i == M) ? cz() : rp;  // I r_p
      scatter(rc, d, i, m, acc);
      fr[0] = m;
    }
    if (i + HW <= M) finish(i + HW);
    shift();
  }
}

hipError_t launch_pc_adj(tc_ctx* c, const cd* ub, const cd* nin, cd* out_u, cd* out_up, cd* out_np, cd* ntot, cd* wA,
                         cd* wH) {
  const int blocks = (c->d.ndm + 31) / 32;
  using K = void (*)(TC_PA_ARGS);
  const K ks[4] = {k_pa1, k_pa2, k_pa3, k_pa4};
  for (const K k : ks) {
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64), 0, c->stream, c->rc_dev, c->fac, c->d, ub, nin, out_u, out_up,
                       out_np, ntot, wA, wH);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace tc
