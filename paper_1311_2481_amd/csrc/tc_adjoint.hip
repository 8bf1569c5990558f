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
//     (mode (0,0): u^{i+1}+- = u*+- - u*_r, so phi_bar = 0 there and
//     u*_bar+- = (u_bar'+- - u_bar'-+)/2)
//   phi = P^-1 div(u*) (interior)    -> r_bar = P^-T phi_bar, u*_bar += div^H(r_bar)
//   u* = H^-1 rhs_u                  -> rhs_u_bar = H^-T u*_bar (interior rows)
//   rhs_u = -(4u - u_prev)/(2dt) + Ne + grad p*
//   p* = P^-1 rhs_p                  -> rp_bar = P^-T grad^H rhs_u_bar
//   rhs_p = -div Ne (interior), -(Ne+ + Ne-)/2 + V_r(2u - u_prev) (walls)
// and the nonlinear term's adjoint (transposed transforms, see the azimuthal
// adjoint kernel) applied to N_bar_total = 2 Ne_bar + N_bar.
//
// The predictor-corrector part runs fused: in four sweeps over the radial
// rows (tc_adjoint_pc.hip), or with each mode's radial line on chip on the
// grids the line kernels take (tc_line.hip).  The nonlinear term's adjoint
// follows: the transposed transforms, then the curl's adjoint below.  On
// small grids it runs one thread per (radial node, stored mode) point, in
// tiles of consecutive slots of one node, numbered node-fastest and walked
// per XCD (see make_slot), and applies D1^T by gathering the (up to 9) rows
// whose stencils touch a node; on large grids one thread per stored mode
// sweeps the radial nodes with those rows in registers.
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

// Work tiles are (radial node k, chunk of SLOT_BLOCK slots), numbered with k
// fastest.  The grid is 1-D with 8 ceil(ntiles / 8) workgroups and
// workgroup b takes tile (b % 8) ceil(ntiles / 8) + b / 8: workgroups are
// dispatched round robin over the 8 XCDs, so each XCD walks a contiguous
// tile range, and the workgroups that need the same slots of neighbouring
// radial planes (the +-4-row stencils) run together and share that XCD's
// L2.  Tiles past the end belong to padding workgroups.
constexpr int SLOT_BLOCK = 256;

__host__ __device__ inline int64_t slot_tiles(const Dims& d) {
  return (d.S + SLOT_BLOCK - 1) / SLOT_BLOCK * (int64_t)d.n_r;
}

// 32-bit index arithmetic: the tile count (at most ceil(S / 256) * 4096) and
// the slot count S of any grid tc_init accepts are far below 2^31, and a
// 64-bit division costs several times a 32-bit one.
__device__ __forceinline__ bool make_slot(const Dims& d, Slot& q) {
  const unsigned ntiles = (unsigned)slot_tiles(d);
  const unsigned per = (ntiles + 7u) / 8u;
  const unsigned id = (blockIdx.x % 8u) * per + blockIdx.x / 8u;
  if (id >= ntiles) return false;
  const unsigned nr = (unsigned)d.n_r, mt = (unsigned)d.mt;
  q.k = (int)(id % nr);
  const unsigned idx = (id / nr) * SLOT_BLOCK + threadIdx.x;
  q.idx = idx;
  if (q.idx >= d.S) return false;
  q.s = (int)(idx / mt);
  q.n = (int)(idx - (unsigned)q.s * mt);
  q.a = q.n * d.kt;
  q.b = (q.s < d.half ? q.s : q.s - d.mz) * d.kz;
  q.nyq = q.s == d.nyq;
  q.zero_mode = q.s == 0 && q.n == 0;
  return true;
}

// (D^T f)_k = sum_i D[i][k] f(i) over the rows i whose stencil touches node
// k, D = D1 (off = RC_W1) or D2 (RC_W2); f(i) is evaluated on the fly, so
// masked or combined fields need no helper array (and no extra pass).
template <class Fn>
__device__ __forceinline__ cd gather_t(const double* rc, const Dims& d, int k, int off, Fn f) {
  cd acc = cz();
  const int M = d.n_r - 1;
  const int lo = k - HW < 0 ? 0 : k - HW, hi = k + HW > M ? M : k + HW;
  for (int i = lo; i <= hi; ++i) {
    const double c = rc[(int64_t)i * RC_N + off + (k - i + HW)];
    const cd v = f(i);
    acc.x = fma(c, v.x, acc.x);
    acc.y = fma(c, v.y, acc.y);
  }
  return acc;
}

}  // namespace

// Curl adjoint: from the direct cotangents (u+d, u-d, u_zd) and those of
// omega (o+, o-, o_z) to the cotangent of (u+, u-, u_z); adds it and
// u_bar_keep into out (which holds the predictor-corrector part).
//   u+  += u+d - b o+ + (i/2) (D1^T o_z + (1+a)/r o_z)
//   u-  += u-d + b o- - (i/2) (D1^T o_z + (1-a)/r o_z)
//   u_z += u_zd - i (a/r)(o+ + o-) + i D1^T (o+ - o-)
__global__ void k_adj_curl(const double* __restrict__ rc, Dims d, const cd* __restrict__ nl,
                           const cd* __restrict__ keep, cd* __restrict__ out) {
  Slot q;
  if (!make_slot(d, q)) return;
  const int64_t F = d.F;
  const cd* upd = nl;
  const cd* umd = nl + F;
  const cd* op = nl + 2 * F;
  const cd* om = nl + 3 * F;
  const cd* uzd = nl + 4 * F;
  const cd* oz = nl + 5 * F;
  const int k = q.k;
  const int64_t o = k * d.S + q.idx;
  if (q.nyq) {
    out[o] = out[F + o] = out[2 * F + o] = cz();
    return;
  }
  const double ir = rc[(int64_t)k * RC_N + RC_IR];
  const cd dz = gather_t(rc, d, k, RC_W1, [&](int i) { return oz[i * d.S + q.idx]; });
  const cd dd = gather_t(rc, d, k, RC_W1, [&](int i) { return cmi(op[i * d.S + q.idx], om[i * d.S + q.idx]); });
  const cd tz_p = cpl(dz, cs(oz[o], (1.0 + q.a) * ir));
  const cd tz_m = cpl(dz, cs(oz[o], (1.0 - q.a) * ir));
  const cd up = cpl(upd[o], cmi(cimul(tz_p, 0.5), cs(op[o], q.b)));
  const cd um = cpl(umd[o], cpl(cs(om[o], q.b), cimul(tz_m, -0.5)));
  const cd uz = cpl(uzd[o], cpl(cimul(cpl(op[o], om[o]), -q.a * ir), cimul(dd, 1.0)));
  out[o] = cpl(out[o], cpl(up, keep[o]));
  out[F + o] = cpl(out[F + o], cpl(um, keep[F + o]));
  out[2 * F + o] = cpl(out[2 * F + o], cpl(uz, keep[2 * F + o]));
}

// The same operation as one radial sweep per stored slot, for large grids:
// a thread walks the nodes of its slot, keeping o+, o- and o_z of the nine
// rows whose stencils reach the current node in registers, so every field
// is read once (the tiled form above gathers o+-, o_z of up to nine rows
// per point through the cache).  The stencil sums run over the rows in the
// same order as gather_t; the two forms agree to rounding (the compiler may
// fuse the remaining products and sums differently in each).
__global__ __launch_bounds__(64) void k_adj_curl_sweep(const double* __restrict__ rc, Dims d,
                                                       const cd* __restrict__ nl, const cd* __restrict__ keep,
                                                       cd* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (idx >= d.S) return;
  const int64_t F = d.F, S = d.S;
  const int M = d.n_r - 1;
  const int s = (int)(idx / d.mt), n = (int)(idx - (int64_t)s * d.mt);
  const double a = n * d.kt;
  const double b = (s < d.half ? s : s - d.mz) * d.kz;
  if (s == d.nyq) {
    for (int k = 0; k <= M; ++k) {
      const int64_t o = k * S + idx;
      out[o] = out[F + o] = out[2 * F + o] = cz();
    }
    return;
  }
  const cd* upd = nl;
  const cd* umd = nl + F;
  const cd* op = nl + 2 * F;
  const cd* om = nl + 3 * F;
  const cd* uzd = nl + 4 * F;
  const cd* oz = nl + 5 * F;
  // window position m holds row k - HW + m
  cd wp[NB9], wm[NB9], wz[NB9];
#pragma unroll
  for (int m = 0; m < NB9; ++m) {
    const int i = m - HW;
    if (i >= 0 && i <= M) {
      wp[m] = op[i * S + idx];
      wm[m] = om[i * S + idx];
      wz[m] = oz[i * S + idx];
    } else {
      wp[m] = wm[m] = wz[m] = cz();
    }
  }
  for (int k = 0; k <= M; ++k) {
    const int64_t o = k * S + idx;
    cd dz = cz(), dd = cz();
#pragma unroll
    for (int m = 0; m < NB9; ++m) {
      const int i = k - HW + m;
      if (i < 0 || i > M) continue;
      const double c = rc[(int64_t)i * RC_N + RC_W1 + (NB9 - 1 - m)];
      const cd vd = cmi(wp[m], wm[m]);
      dz.x = fma(c, wz[m].x, dz.x);
      dz.y = fma(c, wz[m].y, dz.y);
      dd.x = fma(c, vd.x, dd.x);
      dd.y = fma(c, vd.y, dd.y);
    }
    const double ir = rc[(int64_t)k * RC_N + RC_IR];
    const cd opk = wp[HW], omk = wm[HW], ozk = wz[HW];
    const cd tz_p = cpl(dz, cs(ozk, (1.0 + a) * ir));
    const cd tz_m = cpl(dz, cs(ozk, (1.0 - a) * ir));
    const cd up = cpl(upd[o], cmi(cimul(tz_p, 0.5), cs(opk, b)));
    const cd um = cpl(umd[o], cpl(cs(omk, b), cimul(tz_m, -0.5)));
    const cd uz = cpl(uzd[o], cpl(cimul(cpl(opk, omk), -a * ir), cimul(dd, 1.0)));
    out[o] = cpl(out[o], cpl(up, keep[o]));
    out[F + o] = cpl(out[F + o], cpl(um, keep[F + o]));
    out[2 * F + o] = cpl(out[2 * F + o], cpl(uz, keep[2 * F + o]));
    // the window moves to rows k+1-HW .. k+1+HW
#pragma unroll
    for (int m = 0; m < NB9 - 1; ++m) {
      wp[m] = wp[m + 1];
      wm[m] = wm[m + 1];
      wz[m] = wz[m + 1];
    }
    const int inew = k + 1 + HW;
    if (inew <= M) {
      wp[NB9 - 1] = op[inew * S + idx];
      wm[NB9 - 1] = om[inew * S + idx];
      wz[NB9 - 1] = oz[inew * S + idx];
    } else {
      wp[NB9 - 1] = wm[NB9 - 1] = wz[NB9 - 1] = cz();
    }
  }
}

}  // namespace tc

using namespace tc;

namespace {

// Work space of the adjoint calls (allocated on first use): AUX_FIELDS
// fields, then the 9-field transform buffer (double).  Fields: 0, the U^T
// sweeps' output (1 field); 1-6, the nonlinear cotangents (6 fields; fields
// 1-3 first hold the Helmholtz U^T outputs); 7-9, N_tot (3 fields).
constexpr int AUX_FIELDS = 10, AUX_NL6 = 1, AUX_NTOT = 7;
tc_status ensure_aux(tc_ctx* c) {
  const Dims& d = c->d;
  const size_t FB = (size_t)d.F * sizeof(cd);
  const size_t inter9 = (size_t)9 * d.pz * d.mt * sizeof(cd) * d.n_r;
  const size_t need = AUX_FIELDS * FB + inter9;
  if (c->aux_bytes >= need) return TC_OK;
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
  return TC_OK;
}

// Transposed nonlinear term: out += N'(u)^T nbar + keep (3 fields each);
// nl6 (6 fields) and inter (9-field transform buffer) are work space.
hipError_t adjoint_nonlinear(tc_ctx* c, const cd* u, const cd* nbar, const cd* keep, cd* out, cd* nl6, void* inter) {
  const Dims& d = c->d;
  const int64_t F = d.F;
  c->omega_fresh = false;  // the context's curl buffer now holds curl(u)
  hipError_t e = launch_curl(c, u, c->omega);
  if (e != hipSuccess) return e;
  ZIo zi{};
  for (int k = 0; k < 3; ++k) {
    zi.src[k] = u + k * F;
    zi.src[3 + k] = c->omega + k * F;
    zi.src[6 + k] = nbar + k * F;
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
  adjoint_field_map(zo);
  e = launch_zinv_io(c, 0, d.n_r, zi, inter, false);
  if (e == hipSuccess) e = launch_theta_adj(c, d.n_r, inter);
  if (e == hipSuccess) e = launch_zfwd_io(c, 0, d.n_r, zo, inter, false);
  if (e != hipSuccess) return e;
  if (c->adj_curl_sweep) {
    hipLaunchKernelGGL(k_adj_curl_sweep, dim3((unsigned)((d.S + 63) / 64)), dim3(64), 0, c->stream, c->rc_dev, d,
                       nl6, keep, out);
  } else {
    const dim3 blk(SLOT_BLOCK), grd((unsigned)(8 * ((slot_tiles(d) + 7) / 8)));
    hipLaunchKernelGGL(k_adj_curl, grd, blk, 0, c->stream, c->rc_dev, d, nl6, keep, out);
  }
  return hipGetLastError();
}

}  // namespace

extern "C" tc_status tc_step_adjoint(tc_ctx* c, const void* fwd, const void* adj_in, void* adj_out) {
  if (!c) return TC_EINVAL;
  if (!fwd || !adj_in || !adj_out) return fail(c, TC_EINVAL, "NULL array");
  if (c->d.form != TC_ROTATIONAL) return fail(c, TC_EINVAL, "the adjoint step is built for the rotational form");
  const Dims& d = c->d;
  const int64_t F = d.F;
  const size_t FB = (size_t)F * sizeof(cd);
  {
    const char* a = static_cast<const char*>(adj_in);
    const char* b = static_cast<const char*>(adj_out);
    if (a < b + 9 * FB && b < a + 9 * FB) return fail(c, TC_EINVAL, "adj_in and adj_out overlap");
  }
  if (tc_status sa = ensure_aux(c); sa != TC_OK) return sa;
  cd* w = c->aux;
  cd* wA = w;                   // 1 field
  cd* nl6 = w + AUX_NL6 * F;    // 6 fields
  cd* wH = nl6;                 // 3 fields, free again before nl6 is written
  cd* ntot = w + AUX_NTOT * F;  // 3 fields
  void* inter = w + AUX_FIELDS * F;

  const cd* u = static_cast<const cd*>(fwd);
  const cd* ubn = static_cast<const cd*>(adj_in);
  const cd* ukeep = ubn + 3 * F;
  const cd* nin = ubn + 6 * F;
  cd* out = static_cast<cd*>(adj_out);
  cd* out_u = out;
  cd* out_up = out + 3 * F;
  cd* out_np = out + 6 * F;

  hipError_t e;
#define TC_TRY(x) \
  do {            \
    e = (x);      \
    if (e != hipSuccess) return hip_check(c, e, "adjoint step"); \
  } while (0)
  // predictor-corrector, transposed, then the nonlinear term, transposed:
  // forward fields u, omega(u) and the cotangent N_tot
  if (c->flin) TC_TRY(launch_pc_adj_line(c, ubn, nin, out_u, out_up, out_np, ntot));
  else TC_TRY(launch_pc_adj(c, ubn, nin, out_u, out_up, out_np, ntot, wA, wH));
  TC_TRY(adjoint_nonlinear(c, u, ntot, ukeep, out_u, nl6, inter));
#undef TC_TRY
  return TC_OK;
}

// Start of the reverse sweep at step 0, whose history is u^{-1} = u^0 and
// N^{-1} = N(u^0): g = u_bar + u_prev_bar + N'(u^0)^T N_bar.
extern "C" tc_status tc_adjoint_initial_history(tc_ctx* c, const void* u0, const void* adj_in, void* g) {
  if (!c) return TC_EINVAL;
  if (!u0 || !adj_in || !g) return fail(c, TC_EINVAL, "NULL array");
  if (c->d.form != TC_ROTATIONAL) return fail(c, TC_EINVAL, "the adjoint step is built for the rotational form");
  const int64_t F = c->d.F;
  const size_t FB = (size_t)F * sizeof(cd);
  {
    const char* a = static_cast<const char*>(adj_in);
    const char* b = static_cast<const char*>(g);
    if (a < b + 3 * FB && b < a + 9 * FB) return fail(c, TC_EINVAL, "adj_in and g overlap");
  }
  if (tc_status sa = ensure_aux(c); sa != TC_OK) return sa;
  const cd* ub = static_cast<const cd*>(adj_in);
  cd* out = static_cast<cd*>(g);
  hipError_t e = hipMemcpyAsync(out, ub, 3 * FB, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = adjoint_nonlinear(c, static_cast<const cd*>(u0), ub + 6 * F, ub + 3 * F, out, c->aux + AUX_NL6 * F,
                          c->aux + AUX_FIELDS * F);
  return hip_check(c, e, "tc_adjoint_initial_history");
}
