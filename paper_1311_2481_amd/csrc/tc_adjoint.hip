// Discrete adjoint of one projection step (reverse mode of tc_step).
//
// The step maps (u^i, u^{i-1}, N^{i-1}) to (u^{i+1}, u^i, N^i) with
//   N^i = N(u^i), Ne = 2 N^i - N^{i-1},
//   u^{i+1} = PC(Ne, u^i, u^{i-1}) + (boundary constants),
// where PC (steps 2-5 of Sec. 3.2) is linear and acts mode by mode.  Under
// the inner product sum Re(conj(x) y) its adjoint is the conjugate
// transpose: transposed banded solves, D1^T stencils, conjugated i*b
// factors.  Reverse order of the forward chain:
//   u^{i+1} = u* - grad phi          -> phi_bar = -grad^H u_bar', u*_bar = u_bar'
//   phi = P^-1 div(u*) (interior)    -> r_bar = P^-T phi_bar, u*_bar += div^H(r_bar)
//   u* = H^-1 rhs_u                  -> rhs_u_bar = H^-T u*_bar (interior rows)
//   rhs_u = -(4u - u_prev)/(2dt) + Ne + grad p*
//   p* = P^-1 rhs_p                  -> rp_bar = P^-T grad^H rhs_u_bar
//   rhs_p = -div Ne (interior), -(Ne+ + Ne-)/2 + V_r(2u - u_prev) (walls)
// and the nonlinear term's adjoint (transposed transforms, see the azimuthal
// adjoint kernel) applied to N_bar_total = 2 Ne_bar + N_bar.
//
// Work decomposition: one thread per (radial node, stored mode) point on a
// 2-D grid (x: mode slot, y: node); D1^T is applied by gathering the (up to
// 9) rows whose stencils touch a node, from fields written by an earlier
// launch.  The banded transposed solves reuse the solve kernels.
#include "tc_internal.h"

namespace tc {

namespace {

__device__ __forceinline__ cd cz() { return cd{0.0, 0.0}; }
__device__ __forceinline__ cd cs(cd v, double w) { return cd{v.x * w, v.y * w}; }
__device__ __forceinline__ cd cimul(cd v, double w) { return cd{-w * v.y, w * v.x}; }  // i w v
__device__ __forceinline__ cd cpl(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd cmi(cd a, cd b) { return cd{a.x - b.x, a.y - b.y}; }

struct Slot {
  int k;        // radial node
  int64_t idx;  // s * m_theta + n
  int s, n;
  double a, b;
  bool nyq, zero_mode;
};

__device__ __forceinline__ bool make_slot(const Dims& d, Slot& q) {
  q.idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  q.k = blockIdx.y;
  if (q.idx >= d.S) return false;
  q.s = (int)(q.idx / d.mt);
  q.n = (int)(q.idx - (int64_t)q.s * d.mt);
  q.a = q.n * d.kt;
  q.b = (q.s < d.half ? q.s : q.s - d.mz) * d.kz;
  q.nyq = q.s == d.nyq;
  q.zero_mode = q.s == 0 && q.n == 0;
  return true;
}

// (D1^T w)_k = sum_i D1[i][k] w_i; (D2^T w)_k likewise.  w is one field.
__device__ __forceinline__ cd d1t(const double* rc, const Dims& d, const cd* w, int64_t idx, int k, int off) {
  cd acc = cz();
  const int M = d.n_r - 1;
  const int lo = k - HW < 0 ? 0 : k - HW, hi = k + HW > M ? M : k + HW;
  for (int i = lo; i <= hi; ++i) {
    const double c = rc[(int64_t)i * RC_N + off + (k - i + HW)];
    const cd v = w[i * d.S + idx];
    acc.x = fma(c, v.x, acc.x);
    acc.y = fma(c, v.y, acc.y);
  }
  return acc;
}

// grad^H v = D1^T (v+ + v-) - (a/r) v+ + (a/r) v- - i b v_z at node k, with
// v+ + v- read through the helper field vsum (= v+ + v-).
__device__ __forceinline__ cd grad_h(const double* rc, const Dims& d, const cd* v, const cd* vsum, const Slot& q,
                                     int k) {
  const int64_t o = k * d.S + q.idx;
  const double ir = rc[(int64_t)k * RC_N + RC_IR];
  cd g = d1t(rc, d, vsum, q.idx, k, RC_W1);
  g = cpl(g, cs(cmi(v[d.F + o], v[o]), q.a * ir));
  g = cmi(g, cimul(v[2 * d.F + o], q.b));
  return g;
}

}  // namespace

// phi_bar = -grad^H(u_bar'), and vsum = u_bar'+ + u_bar'- (work field).
__global__ void k_adj_phi(const double* __restrict__ rc, Dims d, const cd* __restrict__ ub, cd* __restrict__ vsum,
                          cd* __restrict__ out, int pass) {
  Slot q;
  if (!make_slot(d, q)) return;
  {
    const int k = q.k;
    const int64_t o = k * d.S + q.idx;
    if (pass == 0) {
      vsum[o] = q.nyq ? cz() : cpl(ub[o], ub[d.F + o]);
    } else {
      const cd g = q.nyq ? cz() : grad_h(rc, d, ub, vsum, q, k);
      out[o] = cd{-g.x, -g.y};
    }
  }
}

// u*_bar = u_bar' + div^H(I r), div^H f = (D1^T f/2 + (1+a) f/(2r), D1^T f/2 + (1-a) f/(2r), -i b f);
// pass 0 stores the interior-masked r into mr (work field).
__global__ void k_adj_ustar(const double* __restrict__ rc, Dims d, const cd* __restrict__ ub, const cd* __restrict__ r,
                            cd* __restrict__ mr, cd* __restrict__ us, int pass) {
  Slot q;
  if (!make_slot(d, q)) return;
  const int M = d.n_r - 1;
  {
    const int k = q.k;
    const int64_t o = k * d.S + q.idx;
    if (pass == 0) {
      mr[o] = (k == 0 || k == M || q.nyq) ? cz() : r[o];
      return;
    }
    if (q.nyq) {
      us[o] = us[d.F + o] = us[2 * d.F + o] = cz();
      return;
    }
    const double ir = rc[(int64_t)k * RC_N + RC_IR];
    const cd f = mr[o];
    const cd dt = cs(d1t(rc, d, mr, q.idx, k, RC_W1), 0.5);
    us[o] = cpl(ub[o], cpl(dt, cs(f, 0.5 * (1.0 + q.a) * ir)));
    us[d.F + o] = cpl(ub[d.F + o], cpl(dt, cs(f, 0.5 * (1.0 - q.a) * ir)));
    us[2 * d.F + o] = cmi(ub[2 * d.F + o], cimul(f, q.b));
  }
}

// From rhs_u_bar (masked to interior rows): u_bar = -(2/dt) r, u_prev_bar = r/(2dt),
// Ne_bar = r, p_bar = grad^H r.  pass 0 masks ru in place and forms vsum.
__global__ void k_adj_rhsu(const double* __restrict__ rc, Dims d, cd* __restrict__ ru, cd* __restrict__ vsum,
                           cd* __restrict__ u_b, cd* __restrict__ up_b, cd* __restrict__ ne_b, cd* __restrict__ p_b,
                           int pass) {
  Slot q;
  if (!make_slot(d, q)) return;
  const int M = d.n_r - 1;
  {
    const int k = q.k;
    const int64_t o = k * d.S + q.idx;
    if (pass == 0) {
      const bool z = (k == 0 || k == M || q.nyq);
      for (int c = 0; c < 3; ++c)
        if (z) ru[c * d.F + o] = cz();
      vsum[o] = z ? cz() : cpl(ru[o], ru[d.F + o]);
      return;
    }
    for (int c = 0; c < 3; ++c) {
      const cd r = ru[c * d.F + o];
      u_b[c * d.F + o] = cs(r, -2.0 / d.dt);
      up_b[c * d.F + o] = cs(r, 0.5 / d.dt);
      ne_b[c * d.F + o] = r;
    }
    p_b[o] = q.nyq ? cz() : grad_h(rc, d, ru, vsum, q, k);
  }
}

// Pressure-RHS adjoint: Ne_bar -= div^H(I rp) and -(W rp)/2 on Ne+-;
// V_r^H(W rp) = ((L+^T w)/2, (L-^T w)/2): u_bar += 2 V, u_prev_bar -= V.
// Also writes N_prev_bar = -Ne_bar and N_tot = 2 Ne_bar + N_bar_in.
// pass 0: mr = I rp, wr = W rp (work fields).
__global__ void k_adj_rhsp(const double* __restrict__ rc, Dims d, const cd* __restrict__ rp, cd* __restrict__ mr,
                           cd* __restrict__ wr, cd* __restrict__ ne_b, cd* __restrict__ u_b, cd* __restrict__ up_b,
                           const cd* __restrict__ n_in, cd* __restrict__ n_prev_b, cd* __restrict__ n_tot, int pass) {
  Slot q;
  if (!make_slot(d, q)) return;
  const int M = d.n_r - 1;
  {
    const int k = q.k;
    const int64_t o = k * d.S + q.idx;
    if (pass == 0) {
      const bool wall = (k == 0 || k == M) && !(k == M && q.zero_mode);
      mr[o] = (k == 0 || k == M || q.nyq) ? cz() : rp[o];
      wr[o] = (wall && !q.nyq) ? rp[o] : cz();
      return;
    }
    const double ir = rc[(int64_t)k * RC_N + RC_IR];
    const double ir2 = rc[(int64_t)k * RC_N + RC_IR2];
    cd ne[3] = {ne_b[o], ne_b[d.F + o], ne_b[2 * d.F + o]};
    if (!q.nyq) {
      const cd f = mr[o];
      const cd dt = cs(d1t(rc, d, mr, q.idx, k, RC_W1), 0.5);
      ne[0] = cmi(ne[0], cpl(dt, cs(f, 0.5 * (1.0 + q.a) * ir)));
      ne[1] = cmi(ne[1], cpl(dt, cs(f, 0.5 * (1.0 - q.a) * ir)));
      ne[2] = cpl(ne[2], cimul(f, q.b));  // -(-i b f)
      const cd w = wr[o];
      ne[0] = cmi(ne[0], cs(w, 0.5));
      ne[1] = cmi(ne[1], cs(w, 0.5));
      // L+-^T w = D2^T w + D1^T(w / r) - (a^2/r^2 + b^2 + (1 +- 2a)/r^2) w
      cd t2 = d1t(rc, d, wr, q.idx, k, RC_W2);
      // D1^T (w/r): gather with the 1/r of the stencil row
      cd t1 = cz();
      {
        const int lo = k - HW < 0 ? 0 : k - HW, hi = k + HW > M ? M : k + HW;
        for (int i = lo; i <= hi; ++i) {
          const double c = rc[(int64_t)i * RC_N + RC_W1 + (k - i + HW)] * rc[(int64_t)i * RC_N + RC_IR];
          const cd v = wr[i * d.S + q.idx];
          t1.x = fma(c, v.x, t1.x);
          t1.y = fma(c, v.y, t1.y);
        }
      }
      const cd base = cpl(t2, t1);
      const double dd = q.a * q.a * ir2 + q.b * q.b;
      const cd vp = cs(cmi(base, cs(w, dd + (1.0 + 2.0 * q.a) * ir2)), 0.5);
      const cd vm = cs(cmi(base, cs(w, dd + (1.0 - 2.0 * q.a) * ir2)), 0.5);
      u_b[o] = cpl(u_b[o], cs(vp, 2.0));
      u_b[d.F + o] = cpl(u_b[d.F + o], cs(vm, 2.0));
      up_b[o] = cmi(up_b[o], vp);
      up_b[d.F + o] = cmi(up_b[d.F + o], vm);
    } else {
      ne[0] = ne[1] = ne[2] = cz();
      for (int c = 0; c < 3; ++c) u_b[c * d.F + o] = up_b[c * d.F + o] = cz();
    }
    for (int c = 0; c < 3; ++c) {
      n_prev_b[c * d.F + o] = cd{-ne[c].x, -ne[c].y};
      n_tot[c * d.F + o] = q.nyq ? cz() : cpl(cs(ne[c], 2.0), n_in[c * d.F + o]);
    }
  }
}

// Curl adjoint: from the direct cotangents (u+d, u-d, u_zd) and those of
// omega (o+, o-, o_z) to the cotangent of (u+, u-, u_z); adds it and
// u_bar_keep into out (which holds the predictor-corrector part).
//   u+  += u+d - b o+ + (i/2) (D1^T o_z + (1+a)/r o_z)
//   u-  += u-d + b o- - (i/2) (D1^T o_z + (1-a)/r o_z)
//   u_z += u_zd - i (a/r)(o+ + o-) + i D1^T (o+ - o-)
// pass 0 forms the helper field od = o+ - o-.
__global__ void k_adj_curl(const double* __restrict__ rc, Dims d, const cd* __restrict__ nl, cd* __restrict__ od,
                           const cd* __restrict__ keep, cd* __restrict__ out, int pass) {
  Slot q;
  if (!make_slot(d, q)) return;
  const int64_t F = d.F;
  const cd* upd = nl;
  const cd* umd = nl + F;
  const cd* op = nl + 2 * F;
  const cd* om = nl + 3 * F;
  const cd* uzd = nl + 4 * F;
  const cd* oz = nl + 5 * F;
  {
    const int k = q.k;
    const int64_t o = k * d.S + q.idx;
    if (pass == 0) {
      od[o] = q.nyq ? cz() : cmi(op[o], om[o]);
      return;
    }
    if (q.nyq) {
      out[o] = out[F + o] = out[2 * F + o] = cz();
      return;
    }
    const double ir = rc[(int64_t)k * RC_N + RC_IR];
    const cd dz = d1t(rc, d, oz, q.idx, k, RC_W1);
    const cd tz_p = cpl(dz, cs(oz[o], (1.0 + q.a) * ir));
    const cd tz_m = cpl(dz, cs(oz[o], (1.0 - q.a) * ir));
    cd up = cpl(upd[o], cmi(cimul(tz_p, 0.5), cs(op[o], q.b)));
    cd um = cpl(umd[o], cpl(cs(om[o], q.b), cimul(tz_m, -0.5)));
    cd uz = cpl(uzd[o], cpl(cimul(cpl(op[o], om[o]), -q.a * ir), cimul(d1t(rc, d, od, q.idx, k, RC_W1), 1.0)));
    out[o] = cpl(out[o], cpl(up, keep[o]));
    out[F + o] = cpl(out[F + o], cpl(um, keep[F + o]));
    out[2 * F + o] = cpl(out[2 * F + o], cpl(uz, keep[2 * F + o]));
  }
}

}  // namespace tc

using namespace tc;

extern "C" tc_status tc_step_adjoint(tc_ctx* c, const void* fwd, const void* adj_in, void* adj_out) {
  if (!c) return TC_EINVAL;
  if (!fwd || !adj_in || !adj_out) return fail(c, TC_EINVAL, "NULL array");
  const Dims& d = c->d;
  const int64_t F = d.F;
  const size_t FB = (size_t)F * sizeof(cd);
  {
    const char* a = static_cast<const char*>(adj_in);
    const char* b = static_cast<const char*>(adj_out);
    if (a < b + 9 * FB && b < a + 9 * FB) return fail(c, TC_EINVAL, "adj_in and adj_out overlap");
  }
  // work space: 20 fields + the 9-field transform buffer (double)
  const int NW = 20;
  const size_t inter9 = (size_t)9 * d.pz * d.mt * sizeof(cd) * d.n_r;
  const size_t need = NW * FB + inter9;
  if (c->aux_bytes < need) {
    if (c->aux) {
      (void)hipFree(c->aux);
      c->bytes -= c->aux_bytes;
      c->aux = nullptr;
      c->aux_bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, TC_ENOMEM, "cannot allocate the adjoint work space");
    }
    c->aux = static_cast<cd*>(p);
    c->aux_bytes = need;
    c->bytes += need;
  }
  cd* w = c->aux;
  cd* vsum = w + 0 * F;
  cd* phib = w + 1 * F;
  cd* rphi = w + 2 * F;
  cd* mr = w + 3 * F;
  cd* wr = w + 4 * F;
  cd* us = w + 5 * F;    // 3
  cd* ru = w + 8 * F;    // 3
  cd* neb = w + 11 * F;  // 3
  cd* pb = w + 14 * F;
  cd* rp = w + 15 * F;
  cd* ntot = w + 16 * F;  // 3 (16..18), then the 6 nonlinear cotangents reuse us/ru
  cd* nl6 = us;           // 6 fields: us (3) + ru (3), free by then
  void* inter = w + NW * F;

  const cd* u = static_cast<const cd*>(fwd);
  const cd* ubn = static_cast<const cd*>(adj_in);
  const cd* ukeep = ubn + 3 * F;
  const cd* nin = ubn + 6 * F;
  cd* out = static_cast<cd*>(adj_out);
  cd* out_u = out;
  cd* out_up = out + 3 * F;
  cd* out_np = out + 6 * F;

  const dim3 blk(256), grd((unsigned)((d.S + 255) / 256), (unsigned)d.n_r);
  hipStream_t st = c->stream;
  hipError_t e;
#define TC_TRY(x) \
  do {            \
    e = (x);      \
    if (e != hipSuccess) return hip_check(c, e, "adjoint step"); \
  } while (0)
  // correction and velocity predictor, transposed
  hipLaunchKernelGGL(k_adj_phi, grd, blk, 0, st, c->rc_dev, d, ubn, vsum, phib, 0);
  hipLaunchKernelGGL(k_adj_phi, grd, blk, 0, st, c->rc_dev, d, ubn, vsum, phib, 1);
  TC_TRY(hipGetLastError());
  TC_TRY(launch_solve_t(c, OP_P, 1, phib, rphi));
  hipLaunchKernelGGL(k_adj_ustar, grd, blk, 0, st, c->rc_dev, d, ubn, rphi, mr, us, 0);
  hipLaunchKernelGGL(k_adj_ustar, grd, blk, 0, st, c->rc_dev, d, ubn, rphi, mr, us, 1);
  TC_TRY(hipGetLastError());
  TC_TRY(launch_solve_t(c, OP_HP, 3, us, ru));
  hipLaunchKernelGGL(k_adj_rhsu, grd, blk, 0, st, c->rc_dev, d, ru, vsum, out_u, out_up, neb, pb, 0);
  hipLaunchKernelGGL(k_adj_rhsu, grd, blk, 0, st, c->rc_dev, d, ru, vsum, out_u, out_up, neb, pb, 1);
  TC_TRY(hipGetLastError());
  // pressure predictor, transposed
  TC_TRY(launch_solve_t(c, OP_P, 1, pb, rp));
  hipLaunchKernelGGL(k_adj_rhsp, grd, blk, 0, st, c->rc_dev, d, rp, mr, wr, neb, out_u, out_up, nin, out_np, ntot, 0);
  hipLaunchKernelGGL(k_adj_rhsp, grd, blk, 0, st, c->rc_dev, d, rp, mr, wr, neb, out_u, out_up, nin, out_np, ntot, 1);
  TC_TRY(hipGetLastError());
  // nonlinear term, transposed: forward fields u, omega(u) and the cotangent N_tot
  TC_TRY(launch_curl(c, u, c->omega));
  ZIo zi{};
  for (int k = 0; k < 3; ++k) {
    zi.src[k] = u + k * F;
    zi.src[3 + k] = c->omega + k * F;
    zi.src[6 + k] = ntot + k * F;
  }
  zi.nfields = 9;
  zi.nf_plane = 9;
  ZIo zo{};
  for (int k = 0; k < 6; ++k) zo.dst[k] = nl6 + k * F;
  zo.nfields = 6;
  zo.nf_plane = 9;
  // the transpose of the forward transform carries its 1/(P_theta P_z)
  zo.scale = 1.0 / ((double)d.pt * (double)d.pz);
  zo.weights = 1;
  TC_TRY(launch_zinv_io(c, 0, d.n_r, zi, inter, false));
  TC_TRY(launch_theta_adj(c, d.n_r, inter));
  TC_TRY(launch_zfwd_io(c, 0, d.n_r, zo, inter, false));
  hipLaunchKernelGGL(k_adj_curl, grd, blk, 0, st, c->rc_dev, d, nl6, vsum, ukeep, out_u, 0);
  hipLaunchKernelGGL(k_adj_curl, grd, blk, 0, st, c->rc_dev, d, nl6, vsum, ukeep, out_u, 1);
  TC_TRY(hipGetLastError());
#undef TC_TRY
  return TC_OK;
}
