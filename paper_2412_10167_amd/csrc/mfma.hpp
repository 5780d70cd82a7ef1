// Wavefront-level matrix-core helpers for gfx950 (CDNA4): one 16x16 output
// tile per accumulator, in the four contraction precisions of the library.
//
// Operand layouts (lane l of a 64-wide wavefront), verified on the device:
//   FP64  v_mfma_f64_16x16x4f64   a = A[l%16][k0 + l/16],  b = B[k0 + l/16][l%16]
//                                 d[v] = D[4v + l/16][l%16]
//   FP32  v_mfma_f32_16x16x4f32   same a, b;  d[v] = D[4(l/16) + v][l%16]
//   BF16/FP16 16x16x32            a[t] = A[l%16][k0 + 8(l/16) + t], b[t] = B[k0 + 8(l/16) + t][l%16]
//                                 d[v] = D[4(l/16) + v][l%16]
// The split forms carry each operand as hi + lo (hi = round(x), lo = round(x - hi))
// and accumulate hi*hi + hi*lo + lo*hi in FP32 (the lo*lo term is dropped).
#pragma once
#include <hip/hip_runtime.h>

namespace tdwp {

enum Prec { kP64 = 0, kP32 = 1, kPBF = 2, kPF16 = 3 };

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

template <int P> struct Mma;

template <> struct Mma<kP64> {
  using acc_t = v4d;
  using frag_t = double;
  using out_t = double;
  static constexpr int KS = 4;
  static constexpr double kUnscale = 1.0;
  __device__ static int row(int l, int v) { return 4 * v + (l >> 4); }
  __device__ static acc_t zero() { return acc_t{0, 0, 0, 0}; }
  template <class F> __device__ static frag_t load_a(const F& A, int k0, int l) {
    return A(l & 15, k0 + (l >> 4));
  }
  template <class F> __device__ static frag_t load_b(const F& B, int k0, int l) {
    return B(k0 + (l >> 4), l & 15);
  }
  __device__ static void mma(acc_t& acc, frag_t a, frag_t b) {
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
};

template <> struct Mma<kP32> {
  using acc_t = v4f;
  using frag_t = float;
  using out_t = float;
  static constexpr int KS = 4;
  static constexpr float kUnscale = 1.0f;
  __device__ static int row(int l, int v) { return 4 * (l >> 4) + v; }
  __device__ static acc_t zero() { return acc_t{0, 0, 0, 0}; }
  template <class F> __device__ static frag_t load_a(const F& A, int k0, int l) {
    return (float)A(l & 15, k0 + (l >> 4));
  }
  template <class F> __device__ static frag_t load_b(const F& B, int k0, int l) {
    return (float)B(k0 + (l >> 4), l & 15);
  }
  __device__ static void mma(acc_t& acc, frag_t a, frag_t b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
};

template <class V, class S> struct SplitFrag {
  V hi, lo;
};

// scale: power of two applied to both operands before the split (keeps FP16
// lo parts out of the subnormal range); results are multiplied by 1/scale^2.
template <class V, class S, class F, bool IS_A>
__device__ inline SplitFrag<V, S> split_load(const F& X, int k0, int l, float scale) {
  SplitFrag<V, S> f;
  const int kb = k0 + 8 * (l >> 4);
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const float x = scale * (IS_A ? (float)X(l & 15, kb + t) : (float)X(kb + t, l & 15));
    const S h = (S)x;
    f.hi[t] = h;
    f.lo[t] = (S)(x - (float)h);
  }
  return f;
}

template <> struct Mma<kPBF> {
  using acc_t = v4f;
  using frag_t = SplitFrag<v8bf, __bf16>;
  using out_t = float;
  static constexpr int KS = 32;
  static constexpr float kUnscale = 1.0f;
  __device__ static int row(int l, int v) { return 4 * (l >> 4) + v; }
  __device__ static acc_t zero() { return acc_t{0, 0, 0, 0}; }
  template <class F> __device__ static frag_t load_a(const F& A, int k0, int l) {
    return split_load<v8bf, __bf16, F, true>(A, k0, l, 1.0f);
  }
  template <class F> __device__ static frag_t load_b(const F& B, int k0, int l) {
    return split_load<v8bf, __bf16, F, false>(B, k0, l, 1.0f);
  }
  __device__ static void mma(acc_t& acc, const frag_t& a, const frag_t& b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, acc, 0, 0, 0);
  }
};

template <> struct Mma<kPF16> {
  using acc_t = v4f;
  using frag_t = SplitFrag<v8h, _Float16>;
  using out_t = float;
  static constexpr int KS = 32;
  static constexpr float kScale = 1024.0f;
  static constexpr float kUnscale = 1.0f / (1024.0f * 1024.0f);
  __device__ static int row(int l, int v) { return 4 * (l >> 4) + v; }
  __device__ static acc_t zero() { return acc_t{0, 0, 0, 0}; }
  template <class F> __device__ static frag_t load_a(const F& A, int k0, int l) {
    return split_load<v8h, _Float16, F, true>(A, k0, l, kScale);
  }
  template <class F> __device__ static frag_t load_b(const F& B, int k0, int l) {
    return split_load<v8h, _Float16, F, false>(B, k0, l, kScale);
  }
  __device__ static void mma(acc_t& acc, const frag_t& a, const frag_t& b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a.lo, b.hi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a.hi, b.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a.hi, b.hi, acc, 0, 0, 0);
  }
};


// Compute-format storage of contraction operands, in LDS and for the operator
// tables: FP64, FP32, or hi/lo planes of bf16 / fp16 (plane stride ps elements).
// Tiles are "k-contiguous": element (row r, contraction index k) at r*ld + k, for
// the A operand (rows = output rows) and for the B operand stored transposed
// (rows = output columns).  Split formats need ld and ps multiples of 8.
template <int P> struct Fmt;

template <> struct Fmt<kP64> {
  using E = double;
  using M = Mma<kP64>;
  static constexpr int PLANES = 1, PAD = 1;
  __device__ static M::frag_t frag(const E* t, int ld, int ps, int l, int k0) {
    (void)ps;
    return t[(l & 15) * ld + k0 + (l >> 4)];
  }
  __device__ static void put(E* t, int ps, int idx, double x) { (void)ps; t[idx] = x; }
  // two consecutive entries (idx even)
  __device__ static void put2(E* t, int ps, int idx, double x0, double x1) {
    (void)ps;
    t[idx] = x0;
    t[idx + 1] = x1;
  }
  __device__ static double get(const E* t, int ps, int idx) { (void)ps; return t[idx]; }
};

template <> struct Fmt<kP32> {
  using E = float;
  using M = Mma<kP32>;
  static constexpr int PLANES = 1, PAD = 1;
  __device__ static M::frag_t frag(const E* t, int ld, int ps, int l, int k0) {
    (void)ps;
    return t[(l & 15) * ld + k0 + (l >> 4)];
  }
  __device__ static void put(E* t, int ps, int idx, double x) { (void)ps; t[idx] = (float)x; }
  __device__ static void put2(E* t, int ps, int idx, double x0, double x1) {
    (void)ps;
    t[idx] = (float)x0;
    t[idx + 1] = (float)x1;
  }
  __device__ static double get(const E* t, int ps, int idx) { (void)ps; return (double)t[idx]; }
};

template <class S, class V, int PR> struct SplitFmt {
  using E = S;
  using M = Mma<PR>;
  static constexpr int PLANES = 2, PAD = 8;
  static constexpr float kScale = PR == kPF16 ? 1024.0f : 1.0f;
  __device__ static typename M::frag_t frag(const E* t, int ld, int ps, int l, int k0) {
    const int off = (l & 15) * ld + k0 + 8 * (l >> 4);
    typename M::frag_t f;
    f.hi = *reinterpret_cast<const V*>(t + off);
    f.lo = *reinterpret_cast<const V*>(t + ps + off);
    return f;
  }
  __device__ static void put(E* t, int ps, int idx, double x) {
    const float v = (float)x * kScale;
    const E h = (E)v;
    t[idx] = h;
    t[ps + idx] = (E)(v - (float)h);
  }
  // two consecutive entries (idx and ps even): one 32-bit store per plane
  __device__ static void put2(E* t, int ps, int idx, double x0, double x1) {
    using V2 = E __attribute__((ext_vector_type(2)));
    const float v0 = (float)x0 * kScale, v1 = (float)x1 * kScale;
    const E h0 = (E)v0, h1 = (E)v1;
    *reinterpret_cast<V2*>(t + idx) = V2{h0, h1};
    *reinterpret_cast<V2*>(t + ps + idx) = V2{(E)(v0 - (float)h0), (E)(v1 - (float)h1)};
  }
  __device__ static double get(const E* t, int ps, int idx) {
    return ((double)(float)t[idx] + (double)(float)t[ps + idx]) / (double)kScale;
  }
};
template <> struct Fmt<kPBF> : SplitFmt<__bf16, v8bf, kPBF> {};
template <> struct Fmt<kPF16> : SplitFmt<_Float16, v8h, kPF16> {};

// Per-precision element type of the H u partial sums kept in HBM between passes.
template <int P> struct HType { using T = float; };
template <> struct HType<kP64> { using T = double; };

__host__ __device__ constexpr int round_up(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace tdwp
