// LDS-resident mixed-radix Stockham FFT for gfx950 (radices 8, 4, 2, 3, 5).
//
// A workgroup transforms NF sequences of length L at once.  Element e of
// sequence f lives at buf[e * NF + f] in LDS, so the NF threads that handle
// the same element of neighbouring sequences touch neighbouring addresses.
// Each sequence is served by TPF threads; thread (t, f) has t in [0, TPF).
//
// Pass with radix R after the radices already applied (their product NS):
// butterfly j in [0, L/R) reads x[j + q L/R], q = 0..R-1, multiplies input q
// by w^(q k L/(NS R)) with k = j mod NS and w = exp(SIGN 2 pi i / L), takes
// the R-point DFT and writes output s to (j / NS) NS R + k + s NS.  After
// the last pass the data is in natural order (Stockham autosort).  Every
// pass stages its inputs in registers between two barriers, so it runs in
// place.  SIGN = +1 is the unnormalised inverse transform of eq. fourier,
// SIGN = -1 the forward one (scaling is left to the caller).
#pragma once
#include <hip/hip_runtime.h>

namespace tc {

template <typename T> struct C2 { T x, y; };

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

// One Stockham pass.  W[e] = exp(-2 pi i e / L) (forward roots).
template <typename T, int L, int NF, int TPF, int SIGN, int R, int NS>
__device__ __forceinline__ void stockham_pass(C2<T>* buf, const C2<T>* __restrict__ W, int t, int f) {
  constexpr int NB = L / R;
  constexpr int PER = (NB + TPF - 1) / TPF;
  C2<T> v[PER][R];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int j = t + p * TPF;
    if (NB % TPF == 0 || j < NB) {
#pragma unroll
      for (int q = 0; q < R; ++q) v[p][q] = buf[(j + q * NB) * NF + f];
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int j = t + p * TPF;
    if (NB % TPF == 0 || j < NB) {
      const int k = j % NS;
      if (NS > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          C2<T> w = W[(q * k * (L / (NS * R))) % L];
          if (SIGN > 0) w.y = -w.y;
          v[p][q] = cmul(v[p][q], w);
        }
      }
      Butterfly<R, SIGN, T>::run(v[p]);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int s = 0; s < R; ++s) buf[(base + s * NS) * NF + f] = v[p][s];
    }
  }
  __syncthreads();
}

template <typename T, int L, int NF, int TPF, int SIGN, int P>
__device__ __forceinline__ void stockham_from(C2<T>* buf, const C2<T>* __restrict__ W, int t, int f) {
  constexpr RadixList rl = make_radices(L);
  static_assert(rl.n > 0, "unsupported transform length");
  if constexpr (P < rl.n) {
    constexpr int R = rl.r[P];
    constexpr int NS = radix_product(rl, P);
    stockham_pass<T, L, NF, TPF, SIGN, R, NS>(buf, W, t, f);
    stockham_from<T, L, NF, TPF, SIGN, P + 1>(buf, W, t, f);
  }
}

// Transform NF sequences of length L held in LDS.  The workgroup must have
// exactly NF * TPF threads, all of which call this (it contains barriers).
template <typename T, int L, int NF, int TPF, int SIGN>
__device__ __forceinline__ void fft_lds(C2<T>* buf, const C2<T>* __restrict__ W, int t, int f) {
  stockham_from<T, L, NF, TPF, SIGN, 0>(buf, W, t, f);
}

}  // namespace tc
