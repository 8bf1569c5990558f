// Internal definitions shared by the translation units of libtc.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tc.h"
#include "tc_fft.h"

namespace tc {

using cd = C2<double>;
using cf = C2<float>;

// Radial stencil half-width (9-point central stencils, Sec. 3.1).
constexpr int HW = 4;
constexpr int NB9 = 2 * HW + 1;

// Per-node constants read by every radial kernel (wave-uniform loads):
// r, 1/r, 1/r^2, D1 row weights (9), D2 row weights (9).  Weight k of
// row j multiplies node j + k - 4 (zero outside the shortened stencil).
constexpr int RC_R = 0, RC_IR = 1, RC_IR2 = 2, RC_W1 = 3, RC_W2 = 12, RC_N = 21;

// Factor storage: fac[op][j][c][dm], dm = |l| * m_theta + n a distinct mode
// (the slots +l and -l share one factorisation).  op 0 = P (pressure and
// correction), factored in ascending row order; ops 1-3 = H+, H-, H_z,
// factored in descending row order.  For row j, in the op's own row order:
//   c = 0..3  first-sweep multipliers of the rows 1..4 places earlier,
//   c = 4     1 / pivot,
//   c = 5..8  second-sweep coefficients of the rows 1..4 places later.
constexpr int NOPS = 4, NFAC = 9;
enum { OP_P = 0, OP_HP = 1, OP_HM = 2, OP_HZ = 3 };

// Predictor-corrector with the radial lines on chip (tc_line.hip), for
// grids of n_r = LINE_RPL * LPS radial nodes with LPS ("lanes per slot") a
// power of two: lane k of a slot's LPS lanes holds rows LINE_RPL k ..
// LINE_RPL k + LINE_RPL - 1.  Its factors (flin) hold the values of fac
// lane-contiguously: for operator op, distinct mode dm and lane k, LINE_Q
// pairs of doubles, pair q at
//   flin[((op * ndm + dm) * LINE_Q + q) * 2 LPS + 2 k + {0, 1}];
// counting the lane's doubles e = 0 .. 2 LINE_Q - 1 in pair order, e < 32
// is first-sweep multiplier c = e % 4 of row LINE_RPL k + e / 4, and
// e = 32 + 5 r + c is the inverse pivot (c = 0) or second-sweep
// coefficient c (c = 1..4) of row LINE_RPL k + r.
constexpr int LINE_RPL = 8, LINE_Q1 = 16, LINE_Q = 36;

// Doubles of the static scratch array of tc_get_diag_noalloc (4 MiB per GPU).
constexpr size_t TC_DIAG_SCRATCH_DOUBLES = (size_t)1 << 19;

// Doubles of the context's reduction buffer (block partials).
constexpr size_t TC_RED_DOUBLES = 4096;

// Launch timing slots (tc_kernel_time).
enum { TK_PC = 0, TK_CURL = 1, TK_ZINV = 2, TK_THETA = 3, TK_ZFWD = 4, TK_N = 5 };

struct KernelTimer {
  std::vector<hipEvent_t> ev;  // pairs
  int used = 0;
  bool open = false;  // a start event is recorded and its end is not
  double ms = 0.0;
  int launches = 0;
};

// Sources / destinations of the axial transform kernels: nfields fields
// taken from (or written to) separate spectral arrays, nf_plane fields per
// radial plane in the transform-layout buffer.  For the forward kernel the
// output is multiplied by scale (and by Hermitian weights when weights = 1).
// zmax (inverse kernel, optional): per batch plane, ZMAX_WORDS words; input
// field k adds its largest |component| (as float bits, a maximum) to word
// zmax_slot[k] of its plane (-1: not recorded).  The words start at zero:
// tc_init clears them, and the forward kernel, given zmax, clears the
// batch's words for the next inverse pass.
constexpr int ZMAX_WORDS = 4;
struct ZIo {
  const C2<double>* src[9];
  C2<double>* dst[9];
  int nfields, nf_plane, weights;
  double scale;
  unsigned int* zmax;
  int zmax_slot[9];
  int mulb[9];  // inverse kernel: input field k is multiplied by i l k_z (its z derivative) when set
  // forward kernel: when use_map is set, output k is transformed from the
  // intermediate's field src_field[k] (else from field k)
  int use_map;
  int src_field[9];
};

struct Dims {
  int n_r, mt, mz, pt, pz, nyq, half, ndm;
  int64_t S;      // m_z * m_theta (one radial plane of one field)
  int64_t F;      // n_r * S (one field)
  double kt, kz, dt, Re_i, Re_o;
  double s0, sM;  // scale of the Neumann rows of P (rows 0 and M)
  int form;       // tc_form of the nonlinear term
};

}  // namespace tc

struct tc_ctx {
  tc_grid g{};
  tc::Dims d{};
  double eta = 0, r_i = 0, r_o = 0;
  hipStream_t stream = nullptr;
  std::vector<double> r;    // host copy of the nodes
  std::vector<double> rc;   // host copy of the per-node constants
  // device data owned by the context
  double* rc_dev = nullptr;
  double* fac = nullptr;
  double* flin = nullptr;    // lane-contiguous copy of fac (line predictor-corrector only)
  bool adj_curl_sweep = false;  // curl adjoint as radial sweeps (large grids; see tc_init)
  tc::cd* tw_t = nullptr;   // exp(-2 pi i e / p_theta)
  tc::cd* tw_z = nullptr;   // exp(-2 pi i e / p_z)
  tc::cf* twf_t = nullptr;
  tc::cf* twf_z = nullptr;
  tc::cd* u = nullptr;       // u^i     (3 fields)
  tc::cd* u_prev = nullptr;  // u^{i-1} (3 fields)
  tc::cd* N_prev = nullptr;  // N^{i-1} (3 fields)
  tc::cd* N_cur = nullptr;   // N^i     (3 fields)
  tc::cd* p = nullptr;       // pressure (1 field)
  tc::cd* omega = nullptr;   // curl work (3 fields)
  bool omega_fresh = false;  // omega holds curl(u) of the current state
  tc::cd* aux = nullptr;     // adjoint work (allocated on first use)
  size_t aux_bytes = 0;
  void* inter = nullptr;     // nonlinear intermediate, batch planes
  unsigned int* zmax = nullptr;  // per-plane field magnitudes (ZMAX_WORDS n_r words)
  double* diag_wr = nullptr;     // trapezoid weight times r on every node
  double* diag_uc = nullptr;     // circular Couette u_theta on every node
  double* red = nullptr;         // block partials of small reductions (TC_RED_DOUBLES)
  int device = -1;               // HIP device the context was created on
  double factor_error = 0.0;     // backward error of the factor check at tc_init
  int batch = 0;
  size_t bytes = 0;
  int64_t steps = 0;
  bool have_p = false;
  bool timing = false;
  tc::KernelTimer timers[tc::TK_N];
  std::string err;
};

namespace tc {

// error helpers
tc_status fail(tc_ctx* c, tc_status s, const std::string& msg);
tc_status hip_check(tc_ctx* c, hipError_t e, const char* what);

// launchers (return hipError_t from hipGetLastError)
// (also fills c->flin when it is allocated)
hipError_t launch_factor(tc_ctx* c, int* bad_dev);
// componentwise backward error of the stored factors on one solve per
// operator and mode (tmp: n_r * 4 * ndm doubles of work space)
hipError_t launch_factor_check(tc_ctx* c, double* tmp, unsigned long long* worst_dev);
// largest backward error tc_init accepts from that check
constexpr double TC_FACTOR_CHECK_MAX = 1e-12;
hipError_t launch_solve(tc_ctx* c, int op, int transposed, const cd* rhs, cd* x);
// transposed solves of nop (1, or 3 starting at OP_HP) operators on
// consecutive fields rhs + k F -> x + k F (x may alias rhs)
hipError_t launch_solve_t(tc_ctx* c, int op0, int nop, const cd* rhs, cd* x);
// omega_out (nullable): where the last sweep also writes curl(u_next) on
// grids where pc_fuses_curl() holds (ignored elsewhere)
hipError_t launch_pc(tc_ctx* c, const cd* u, const cd* u_prev, const cd* N, cd* N_prev_scratch,
                     cd* u_next, cd* p, int want_p, cd* omega_out);
bool pc_fuses_curl(const tc_ctx* c);
// the line predictor-corrector (tc_line.hip): its lanes per slot on this
// grid (0 where it does not run), and its launch (the arguments of
// launch_pc; omg NULL: no curl)
int line_lps(const Dims& d);
hipError_t launch_pc_line(tc_ctx* c, const cd* u, const cd* u_prev, const cd* N, const cd* N_prev, cd* u_next,
                          cd* p, int want_p, cd* omg);
// transposed solves on the line layout (the arguments of launch_solve_t)
hipError_t launch_solve_t_line(tc_ctx* c, int op0, int nop, const cd* rhs, cd* x);
// the adjoint step's predictor-corrector part on the line layout: from the
// cotangents of u^{i+1} (ub) and N^i (nin) to those of u^i (out_u, before
// the nonlinear term's part), u^{i-1}, N^{i-1} and the total cotangent of
// N(u^i) (ntot); 3 fields each
hipError_t launch_pc_adj_line(tc_ctx* c, const cd* ub, const cd* nin, cd* out_u, cd* out_up, cd* out_np, cd* ntot);
// the same in four sweeps (tc_adjoint_pc.hip), for the other grids; wA (1
// field) and wH (3 fields) are work space
hipError_t launch_pc_adj(tc_ctx* c, const cd* ub, const cd* nin, cd* out_u, cd* out_up, cd* out_np, cd* ntot, cd* wA,
                         cd* wH);
hipError_t launch_curl(tc_ctx* c, const cd* u, cd* omega);
hipError_t launch_zinv(tc_ctx* c, int plane0, int nplanes, const cd* u, const cd* omega);
hipError_t launch_theta(tc_ctx* c, int nplanes);
hipError_t launch_zfwd(tc_ctx* c, int plane0, int nplanes, cd* N);
hipError_t launch_zinv_io(tc_ctx* c, int plane0, int np, const ZIo& io, void* inter, bool f32);
hipError_t launch_zfwd_io(tc_ctx* c, int plane0, int np, const ZIo& io, const void* inter, bool f32);
hipError_t launch_theta_adj(tc_ctx* c, int nplanes, void* inter);
// which intermediate fields the axial forward pass of the adjoint reads
// (where the azimuthal adjoint kernel leaves its six results)
void adjoint_field_map(ZIo& zo);
// convective form: radial derivatives D1 u (3 fields) and the azimuthal
// pass over the 9-field intermediate of planes plane0 ..
hipError_t launch_dr(tc_ctx* c, const cd* u, cd* du);
hipError_t launch_zinv_conv(tc_ctx* c, int plane0, int nplanes, const cd* u, const cd* du);
hipError_t launch_theta_conv(tc_ctx* c, int plane0, int nplanes);
int inter_fields(const tc_ctx* c);
bool fft_length_supported(int L);
size_t inter_bytes_per_plane(const tc_ctx* c);

// kinetic energy 1/2 int |u|^2 dV of a velocity (synchronous; uses ctx->red)
hipError_t energy_of(tc_ctx* c, const cd* u, double& E);

// timing helpers (no-ops unless ctx->timing)
void timer_begin(tc_ctx* c, int which);
void timer_end(tc_ctx* c, int which);

}  // namespace tc
