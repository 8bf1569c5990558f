// Mixed-radix Stockham FFT for gfx950 (radices 8, 4, 2, 3, 5), registers
// plus LDS exchanges.
//
// A workgroup transforms NF sequences of length L at once, TPF threads per
// sequence; thread (t, f) has t in [0, TPF), f in [0, NF).
//
// Pass with radix R after the radices already applied (their product NS):
// butterfly j in [0, L/R) reads x[j + q L/R], q = 0..R-1, multiplies input q
// by w^(q k L/(NS R)) with k = j mod NS and w = exp(SIGN 2 pi i / L), takes
// the R-point DFT and writes output s to (j / NS) NS R + k + s NS.  After
// the last pass the data is in natural order (Stockham autosort).
// Butterfly j of every pass belongs to thread t = j mod TPF.
//
// The first pass takes its inputs from registers filled by the caller
// (element j + q L/R0 in slot [k][q], j = t + k TPF), the last pass leaves
// its outputs in registers (element j + s L/RN in slot [k][s]): only the
// exchanges between passes go through LDS.  A transform run with the radix
// order reversed starts exactly where a transform in natural order ends
// (its first-pass inputs are the other's last-pass outputs in the same
// slots), so a pointwise product between an inverse and a forward
// transform never leaves registers.
//
// LDS layout: element e of sequence f at (e + e/8) * NF + f; the pad word
// every 8 elements spreads the stride-8 writes of the early passes over
// the banks.  SIGN = +1 is the unnormalised inverse transform of eq.
// fourier, SIGN = -1 the forward one (scaling is left to the caller).
#pragma once
#include <hip/hip_runtime.h>

namespace tc {

// Aligned to its full size so that LDS and global accesses are single
// 128-bit (double) or 64-bit (float) operations: split 64-bit accesses of
// interleaved complex data would hit the LDS banks two-way.
template <typename T> struct alignas(2 * sizeof(T)) C2 { T x, y; };

template <typename T> __device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by SIGN * i
template <int SIGN, typename T> __device__ __forceinline__ C2<T> mul_si(C2<T> a) {
  return SIGN > 0 ? C2<T>{-a.y, a.x} : C2<T>{a.y, -a.x};
}
template <typename T> __device__ __forceinline__ C2<T> cconj(C2<T> a) { return {a.x, -a.y}; }

struct RadixList {
  int n;
  int r[24];
};

constexpr RadixList make_radices(int L) {
  RadixList rl{0, {}};
  while (L % 8 == 0) { rl.r[rl.n++] = 8; L /= 8; }
  while (L % 4 == 0) { rl.r[rl.n++] = 4; L /= 4; }
  while (L % 2 == 0) { rl.r[rl.n++] = 2; L /= 2; }
  while (L % 3 == 0) { rl.r[rl.n++] = 3; L /= 3; }
  while (L % 5 == 0) { rl.r[rl.n++] = 5; L /= 5; }
  if (L != 1) rl.n = -1;
  return rl;
}

constexpr int radix_product(const RadixList& rl, int upto) {
  int p = 1;
  for (int i = 0; i < upto; ++i) p *= rl.r[i];
  return p;
}

// R-point DFT in registers, y_s = sum_q v_q exp(SIGN 2 pi i q s / R).
template <int R, int SIGN, typename T> struct Butterfly;

template <int SIGN, typename T> struct Butterfly<2, SIGN, T> {
  static __device__ __forceinline__ void run(C2<T>* v) {
    C2<T> a = cadd(v[0], v[1]), b = csub(v[0], v[1]);
    v[0] = a; v[1] = b;
  }
};

template <int SIGN, typename T> struct Butterfly<4, SIGN, T> {
  static __device__ __forceinline__ void run(C2<T>* v) {
    C2<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    C2<T> t2 = cadd(v[1], v[3]), t3 = mul_si<SIGN>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2); v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3); v[3] = csub(t1, t3);
  }
};

template <int SIGN, typename T> struct Butterfly<8, SIGN, T> {
  static __device__ __forceinline__ void run(C2<T>* v) {
    C2<T> e[4] = {v[0], v[2], v[4], v[6]};
    C2<T> o[4] = {v[1], v[3], v[5], v[7]};
    Butterfly<4, SIGN, T>::run(e);
    Butterfly<4, SIGN, T>::run(o);
    const T h = T(0.70710678118654752440084436210484903928);
    // o_k *= exp(SIGN 2 pi i k / 8)
    C2<T> o1 = {h * (o[1].x - T(SIGN) * o[1].y), h * (o[1].y + T(SIGN) * o[1].x)};
    C2<T> o2 = mul_si<SIGN>(o[2]);
    C2<T> o3 = {h * (-o[3].x - T(SIGN) * o[3].y), h * (-o[3].y + T(SIGN) * o[3].x)};
    v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
  }
};

template <int SIGN, typename T> struct Butterfly<3, SIGN, T> {
  static __device__ __forceinline__ void run(C2<T>* v) {
    const T s3 = T(0.86602540378443864676372317075293618347);
    C2<T> a = cadd(v[1], v[2]);
    C2<T> d = csub(v[1], v[2]);
    C2<T> t = {v[0].x - T(0.5) * a.x, v[0].y - T(0.5) * a.y};
    C2<T> s = mul_si<SIGN>(cscale(d, s3));
    v[0] = cadd(v[0], a);
    v[1] = cadd(t, s);
    v[2] = csub(t, s);
  }
};

template <int SIGN, typename T> struct Butterfly<5, SIGN, T> {
  static __device__ __forceinline__ void run(C2<T>* v) {
    const T c1 = T(0.30901699437494742410229341718281905886);
    const T c2 = T(-0.80901699437494742410229341718281905886);
    const T s1 = T(0.95105651629515357211643933337938214340);
    const T s2 = T(0.58778525229247312916870595463907276860);
    C2<T> a1 = cadd(v[1], v[4]), a2 = cadd(v[2], v[3]);
    C2<T> b1 = csub(v[1], v[4]), b2 = csub(v[2], v[3]);
    C2<T> t1 = {v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y};
    C2<T> t2 = {v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y};
    C2<T> u1 = mul_si<SIGN>(C2<T>{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
    C2<T> u2 = mul_si<SIGN>(C2<T>{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(t1, u1); v[4] = csub(t1, u1);
    v[2] = cadd(t2, u2); v[3] = csub(t2, u2);
  }
};


constexpr RadixList reversed(RadixList rl) {
  RadixList o{rl.n, {}};
  for (int i = 0; i < rl.n; ++i) o.r[i] = rl.r[rl.n - 1 - i];
  return o;
}

// LDS slot of element e.  SWZ = false: one pad word every 8 elements.
// SWZ = true (lengths that are multiples of 16): no padding; the slots of
// each 16-element block are permuted by bits 3-6 and 9-12 of e, which
// removes the bank conflicts of the strided exchanges at the cost of a few
// integer operations per access.
template <int L, bool SWZ> __host__ __device__ constexpr int lds_slot(int e) {
  if constexpr (SWZ) {
    static_assert(L % 16 == 0, "swizzled layout needs L % 16 == 0");
    return (e & ~15) | ((e ^ (e >> 3) ^ (e >> 9)) & 15);
  } else {
    return e + (e >> 3);
  }
}
template <int L, bool SWZ> __host__ __device__ constexpr int lds_len() {
  if constexpr (SWZ) return L;
  else return lds_slot<L, false>(L - 1) + 1;
}

// Twiddles w^q, q = 1..R-1, of one butterfly, w = W[base] (conjugated for
// SIGN > 0).  With TC_TW_DERIVE only w, w^2 (and w^4 for radix 8) are
// loaded and the other powers formed by complex products (a few ulp).
#ifndef TC_TW_DERIVE
#define TC_TW_DERIVE 1
#endif
template <int R, int SIGN, typename T>
__device__ __forceinline__ void twiddles(const C2<T>* __restrict__ W, int base, C2<T>* w) {
  auto ld = [&](int q) {
    C2<T> x = W[q * base];
    if (SIGN > 0) x.y = -x.y;
    return x;
  };
  if constexpr (!TC_TW_DERIVE || R == 2) {
#pragma unroll
    for (int q = 1; q < R; ++q) w[q] = ld(q);
  } else if constexpr (R == 3) {
    w[1] = ld(1);
    w[2] = cmul(w[1], w[1]);
  } else if constexpr (R == 4) {
    w[1] = ld(1);
    w[2] = ld(2);
    w[3] = cmul(w[1], w[2]);
  } else if constexpr (R == 5) {
    w[1] = ld(1);
    w[2] = ld(2);
    w[3] = cmul(w[1], w[2]);
    w[4] = cmul(w[2], w[2]);
  } else {
    static_assert(R == 8, "radix");
    w[1] = ld(1);
    w[2] = ld(2);
    w[4] = ld(4);
    w[3] = cmul(w[1], w[2]);
    w[5] = cmul(w[1], w[4]);
    w[6] = cmul(w[2], w[4]);
    w[7] = cmul(w[3], w[4]);
  }
}

// v[q] *= w^q, q = 1..R-1.  In double with TC_TW_CHAIN the powers are formed
// one after another (w^q = w^(q-1) w, a few ulp), so that only two twiddles
// are live: register pressure decides the occupancy of the long transforms.
#ifndef TC_TW_CHAIN
#define TC_TW_CHAIN 1
#endif
template <int R, int SIGN, typename T>
__device__ __forceinline__ void apply_twiddles(const C2<T>* __restrict__ W, int base, C2<T>* v) {
  if constexpr (TC_TW_CHAIN && sizeof(T) == 8 && R > 2) {
    C2<T> w1 = W[base];
    if (SIGN > 0) w1.y = -w1.y;
    C2<T> wq = w1;
    v[1] = cmul(v[1], w1);
#pragma unroll
    for (int q = 2; q < R; ++q) {
      wq = cmul(wq, w1);
      v[q] = cmul(v[q], wq);
    }
  } else {
    C2<T> w[R];
    twiddles<R, SIGN, T>(W, base, w);
#pragma unroll
    for (int q = 1; q < R; ++q) v[q] = cmul(v[q], w[q]);
  }
}

template <typename T, int L, int TPF, int SIGN, bool REV, bool SWZ = false>
struct Fft {
  static constexpr RadixList RL = REV ? reversed(make_radices(L)) : make_radices(L);
  static_assert(RL.n > 0, "unsupported transform length");
  static constexpr int P = RL.n;
  static constexpr int R0 = RL.r[0];
  static constexpr int RN = RL.r[P - 1];
  static constexpr int PER0 = (L / R0 + TPF - 1) / TPF;
  static constexpr int PERN = (L / RN + TPF - 1) / TPF;
  using In = C2<T>[PER0][R0];
  using Out = C2<T>[PERN][RN];

  // middle pass P0 (0 < P0 < P-1): LDS src -> LDS dst
  template <int NF, int PP>
  static __device__ __forceinline__ void mid(const C2<T>* src, C2<T>* dst, const C2<T>* __restrict__ W, int t, int f,
                                             bool inplace) {
    constexpr int R = RL.r[PP];
    constexpr int NS = radix_product(RL, PP);
    constexpr int NB = L / R;
    constexpr int PER = (NB + TPF - 1) / TPF;
    C2<T> v[PER][R];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int j = t + k * TPF;
      if (NB % TPF == 0 || j < NB) {
#pragma unroll
        for (int q = 0; q < R; ++q) v[k][q] = src[lds_slot<L, SWZ>(j + q * NB) * NF + f];
      }
    }
    if (inplace) __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int j = t + k * TPF;
      if (NB % TPF == 0 || j < NB) {
        const int kk = j % NS;
        apply_twiddles<R, SIGN, T>(W, kk * (L / (NS * R)), v[k]);  // q kk L/(NS R) < L
        Butterfly<R, SIGN, T>::run(v[k]);
        const int base = (j / NS) * NS * R + kk;
#pragma unroll
        for (int s = 0; s < R; ++s) dst[lds_slot<L, SWZ>(base + s * NS) * NF + f] = v[k][s];
      }
    }
    __syncthreads();
  }

  template <int NF, int PP>
  static __device__ __forceinline__ void mids(C2<T>* a, C2<T>* b, const C2<T>* __restrict__ W, int t, int f,
                                              bool inplace) {
    if constexpr (PP < P - 1) {
      mid<NF, PP>(a, b, W, t, f, inplace);
      mids<NF, PP + 1>(b, a, W, t, f, inplace);
    }
  }

  // buffer the data ends in after the middle passes (for the last pass)
  static constexpr bool ENDS_IN_B = ((P - 2) % 2) == 1;

  // Full transform.  a, b: LDS buffers of lds_len<L>() * NF elements each
  // (b may equal a: in-place mode, two barriers per exchange).  Ends with a
  // barrier, so the buffers may be reused at once.
  template <int NF>
  static __device__ __forceinline__ void run(In& v0, Out& vn, C2<T>* a, C2<T>* b, const C2<T>* __restrict__ W, int t,
                                             int f) {
    const bool inplace = (a == b);
    if constexpr (P == 1) {
#pragma unroll
      for (int k = 0; k < PER0; ++k) {
        Butterfly<R0, SIGN, T>::run(v0[k]);
#pragma unroll
        for (int s = 0; s < R0; ++s) vn[k][s] = v0[k][s];
      }
      return;
    } else {
      // first pass: NS = 1, no twiddles; outputs j R0 + s
      {
        constexpr int NB = L / R0;
#pragma unroll
        for (int k = 0; k < PER0; ++k) {
          const int j = t + k * TPF;
          if (NB % TPF == 0 || j < NB) {
            Butterfly<R0, SIGN, T>::run(v0[k]);
#pragma unroll
            for (int s = 0; s < R0; ++s) a[lds_slot<L, SWZ>(j * R0 + s) * NF + f] = v0[k][s];
          }
        }
        __syncthreads();
      }
      mids<NF, 1>(a, b, W, t, f, inplace);
      // last pass: NS = L / RN; outputs j + s L/RN
      {
        const C2<T>* src = ENDS_IN_B ? b : a;
        constexpr int NS = L / RN;
        constexpr int NB = L / RN;
#pragma unroll
        for (int k = 0; k < PERN; ++k) {
          const int j = t + k * TPF;
          if (NB % TPF == 0 || j < NB) {
#pragma unroll
            for (int q = 0; q < RN; ++q) vn[k][q] = src[lds_slot<L, SWZ>(j + q * NB) * NF + f];
            apply_twiddles<RN, SIGN, T>(W, j * (L / (NS * RN)), vn[k]);
            Butterfly<RN, SIGN, T>::run(vn[k]);
          }
        }
        __syncthreads();
      }
    }
  }

  // The same transform with each LDS exchange done one component at a time
  // through a buffer of T (half the bytes of the complex buffer): the real
  // parts are written in this pass's output order and read in the next
  // pass's input order, then the imaginary parts.  Four barriers per
  // exchange instead of two, for half the LDS.  v: the inputs of pass PP
  // (element j + q L/R, j = t + k TPF); buf: lds_len<L>() * NF elements.
  template <int NF, int PP, int PER, int R>
  static __device__ __forceinline__ void pass_split(C2<T> (&v)[PER][R], Out& vn, T* buf, const C2<T>* __restrict__ W,
                                                    int t, int f) {
    constexpr int NS = radix_product(RL, PP);
    constexpr int NB = L / R;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int j = t + k * TPF;
      if (NB % TPF == 0 || j < NB) {
        if constexpr (PP > 0) apply_twiddles<R, SIGN, T>(W, (j % NS) * (L / (NS * R)), v[k]);
        Butterfly<R, SIGN, T>::run(v[k]);
      }
    }
    if constexpr (PP == P - 1) {
#pragma unroll
      for (int k = 0; k < PER; ++k)
#pragma unroll
        for (int s = 0; s < R; ++s) vn[k][s] = v[k][s];
    } else {
      constexpr int R2 = RL.r[PP + 1];
      constexpr int NB2 = L / R2;
      constexpr int PER2 = (NB2 + TPF - 1) / TPF;
      C2<T> nx[PER2][R2];
#pragma unroll
      for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int j = t + k * TPF;
          if (NB % TPF == 0 || j < NB) {
            const int base = (j / NS) * NS * R + j % NS;
#pragma unroll
            for (int s = 0; s < R; ++s) buf[lds_slot<L, SWZ>(base + s * NS) * NF + f] = comp ? v[k][s].y : v[k][s].x;
          }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER2; ++k) {
          const int j = t + k * TPF;
          if (NB2 % TPF == 0 || j < NB2) {
#pragma unroll
            for (int q = 0; q < R2; ++q) {
              const T x = buf[lds_slot<L, SWZ>(j + q * NB2) * NF + f];
              if (comp) nx[k][q].y = x;
              else nx[k][q].x = x;
            }
          }
        }
        __syncthreads();
      }
      pass_split<NF, PP + 1, PER2, R2>(nx, vn, buf, W, t, f);
    }
  }
  template <int NF>
  static __device__ __forceinline__ void run_split(In& v0, Out& vn, T* buf, const C2<T>* __restrict__ W, int t,
                                                   int f) {
    pass_split<NF, 0, PER0, R0>(v0, vn, buf, W, t, f);
  }

  // element index held in register slot [k][q] before / after the transform
  static __device__ __forceinline__ int in_index(int t, int k, int q) { return t + k * TPF + q * (L / R0); }
  static __device__ __forceinline__ int out_index(int t, int k, int s) { return t + k * TPF + s * (L / RN); }
  static __device__ __forceinline__ bool in_valid(int t, int k) { return (L / R0) % TPF == 0 || t + k * TPF < L / R0; }
  static __device__ __forceinline__ bool out_valid(int t, int k) { return (L / RN) % TPF == 0 || t + k * TPF < L / RN; }
};

}  // namespace tc
