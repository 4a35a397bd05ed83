// Device FFT building blocks for gfx950 (wave64).
//
// A length-L transform is computed by T cooperating threads, each holding
// E = L / T complex values in registers.  Thread t always holds the elements
// at positions t + T*i (i = 0..E-1): on entry those are the inputs in natural
// order, on exit the outputs in natural order.  The passes follow the
// Stockham autosort scheme (each radix-R pass reads elements j + r L/R and
// writes the butterfly outputs to (j / s) s R + (j mod s) + r s, s being the
// product of the earlier radices), so no bit reversal is needed; between
// passes the values are exchanged through LDS.  With the t + T*i register
// layout the last pass writes exactly the positions its thread holds, so a
// transform of P passes needs P - 1 LDS exchanges.
//
// Twiddles come from per-pass tables computed on the host in FP64 and rounded
// once to FP32 (no device sin/cos, no recurrences); radix-4 passes hold them
// as (cosine, tangent) pairs for a fused multiply-add butterfly.  The
// small in-register DFTs use exact radix-2/4 forms, radix-3/5 forms with
// FP64-rounded constants, Good-Thomas splits for coprime composites and a
// Cooley-Tukey split with constant twiddles for 8 and 16.
#pragma once

#include <hip/hip_runtime.h>

namespace litho {
namespace dev {

typedef float2 cf;

__device__ __forceinline__ cf cmake(float x, float y) { return make_float2(x, y); }
__device__ __forceinline__ cf cadd(cf a, cf b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cf csub(cf a, cf b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cf cscale(cf a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ cf cmul(cf a, cf b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ cf cconj(cf a) { return make_float2(a.x, -a.y); }
// a * conj(b)
__device__ __forceinline__ cf cmulc(cf a, cf b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float cabs2(cf a) { return a.x * a.x + a.y * a.y; }
// a * (DIR * i):  i (x + iy) = -y + ix
template <int DIR>
__device__ __forceinline__ cf cmul_i(cf a) {
  return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// cos / sin of 2 pi m / 16, m = 0..15 (exact values rounded to float).
__device__ constexpr float kCos16[16] = {
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
__device__ constexpr float kSin16[16] = {
    0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
    1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
    0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
    -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};

// a * exp(DIR * 2 pi i m / 16) with the trivial angles folded at compile time.
template <int M, int DIR>
__device__ __forceinline__ cf twiddle16(cf a) {
  constexpr int m = ((M % 16) + 16) % 16;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (m == 4) {
    return cmul_i<DIR>(a);
  } else if constexpr (m == 8) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (m == 12) {
    return cmul_i<-DIR>(a);
  } else {
    const float c = kCos16[m];
    const float s = DIR > 0 ? kSin16[m] : -kSin16[m];
    return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
  }
}

// ------------------------------------------------------------------ small DFTs
// Dft<R, DIR>::run(v): in-place X[k] = sum_n v[n] exp(DIR 2 pi i n k / R).
template <int R, int DIR>
struct Dft;

template <int DIR>
struct Dft<1, DIR> {
  __device__ __forceinline__ static void run(cf *) {}
};

template <int DIR>
struct Dft<2, DIR> {
  __device__ __forceinline__ static void run(cf *v) {
    const cf a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
  }
};

template <int DIR>
struct Dft<3, DIR> {
  __device__ __forceinline__ static void run(cf *v) {
    constexpr float s3 = 0.86602540378443865f;  // sin(2 pi / 3)
    const cf t1 = cadd(v[1], v[2]);
    const cf t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
    const cf t3 = cmul_i<DIR>(cscale(csub(v[1], v[2]), s3));
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
  }
};

template <int DIR>
struct Dft<4, DIR> {
  __device__ __forceinline__ static void run(cf *v) {
    const cf a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    const cf c = cadd(v[1], v[3]), d = cmul_i<DIR>(csub(v[1], v[3]));
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  }
};

template <int DIR>
struct Dft<5, DIR> {
  __device__ __forceinline__ static void run(cf *v) {
    constexpr float c1 = 0.30901699437494742f;   // cos(2 pi / 5)
    constexpr float c2 = -0.80901699437494742f;  // cos(4 pi / 5)
    constexpr float s1 = 0.95105651629515357f;   // sin(2 pi / 5)
    constexpr float s2 = 0.58778525229247313f;   // sin(4 pi / 5)
    const cf a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const cf a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const cf x0 = v[0];
    const cf p1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
    const cf p2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
    const cf q1 = cmul_i<DIR>(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
    const cf q2 = cmul_i<DIR>(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
    v[0] = cadd(x0, cadd(a1, a2));
    v[1] = cadd(p1, q1);
    v[4] = csub(p1, q1);
    v[2] = cadd(p2, q2);
    v[3] = csub(p2, q2);
  }
};

constexpr int ct_gcd(int a, int b) { return b == 0 ? a : ct_gcd(b, a % b); }
constexpr int ct_inv_mod(int a, int m) {  // a^-1 mod m for gcd(a, m) = 1, m >= 1
  int r = 0;
  for (int x = 0; x < m; ++x)
    if ((a * x) % m == 1 % m) r = x;
  return r;
}

// Good-Thomas split R = A * B, gcd(A, B) = 1: no twiddles.
// input n = (B n1 + A n2) mod R, output k = CRT(k1 mod A, k2 mod B).
template <int A, int B, int DIR>
struct DftPfa {
  static_assert(ct_gcd(A, B) == 1, "coprime factors required");
  __device__ __forceinline__ static void run(cf *v) {
    constexpr int R = A * B;
    cf t[B][A];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2)
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) t[n2][n1] = v[(B * n1 + A * n2) % R];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) Dft<A, DIR>::run(t[n2]);
    cf u[A][B];
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1)
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) u[k1][n2] = t[n2][k1];
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) Dft<B, DIR>::run(u[k1]);
    constexpr int eA = B * ct_inv_mod(B % A, A);
    constexpr int eB = A * ct_inv_mod(A % B, B);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1)
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) v[(k1 * eA + k2 * eB) % R] = u[k1][k2];
  }
};

// Cooley-Tukey split R = A * B (R divides 16): n = B n1 + n2, k = k1 + A k2,
// twiddle exp(DIR 2 pi i n2 k1 / R) between the A-point and B-point stages.
template <int A, int B, int DIR>
struct DftCt {
  __device__ __forceinline__ static void run(cf *v) {
    constexpr int R = A * B;
    static_assert(16 % R == 0, "constant twiddles cover divisors of 16");
    cf t[B][A];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) t[n2][n1] = v[B * n1 + n2];
      Dft<A, DIR>::run(t[n2]);
    }
    cf u[A][B];
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) {
        const int m = (n2 * k1) * (16 / R);
        // m is a compile-time constant after unrolling
        u[k1][n2] = t[n2][k1];
        switch (m) {  // folded by the compiler
          case 0: break;
          case 1: u[k1][n2] = twiddle16<1, DIR>(u[k1][n2]); break;
          case 2: u[k1][n2] = twiddle16<2, DIR>(u[k1][n2]); break;
          case 3: u[k1][n2] = twiddle16<3, DIR>(u[k1][n2]); break;
          case 4: u[k1][n2] = twiddle16<4, DIR>(u[k1][n2]); break;
          case 5: u[k1][n2] = twiddle16<5, DIR>(u[k1][n2]); break;
          case 6: u[k1][n2] = twiddle16<6, DIR>(u[k1][n2]); break;
          case 7: u[k1][n2] = twiddle16<7, DIR>(u[k1][n2]); break;
          case 8: u[k1][n2] = twiddle16<8, DIR>(u[k1][n2]); break;
          case 9: u[k1][n2] = twiddle16<9, DIR>(u[k1][n2]); break;
          case 10: u[k1][n2] = twiddle16<10, DIR>(u[k1][n2]); break;
          case 11: u[k1][n2] = twiddle16<11, DIR>(u[k1][n2]); break;
          case 12: u[k1][n2] = twiddle16<12, DIR>(u[k1][n2]); break;
          case 13: u[k1][n2] = twiddle16<13, DIR>(u[k1][n2]); break;
          case 14: u[k1][n2] = twiddle16<14, DIR>(u[k1][n2]); break;
          default: u[k1][n2] = twiddle16<15, DIR>(u[k1][n2]); break;
        }
      }
      Dft<B, DIR>::run(u[k1]);
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1)
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = u[k1][k2];
  }
};

template <int DIR> struct Dft<6, DIR> : DftPfa<2, 3, DIR> {};
template <int DIR> struct Dft<8, DIR> : DftCt<2, 4, DIR> {};
template <int DIR> struct Dft<10, DIR> : DftPfa<2, 5, DIR> {};
template <int DIR> struct Dft<12, DIR> : DftPfa<4, 3, DIR> {};
template <int DIR> struct Dft<16, DIR> : DftCt<4, 4, DIR> {};
template <int DIR> struct Dft<20, DIR> : DftPfa<4, 5, DIR> {};

// ------------------------------------------------------------------ plans
template <int... Rs>
struct Radices {};

// FftPlan<L>: threads per transform T and the radix sequence (each radix must
// divide E = L / T; their product is L).
template <int L>
struct FftPlan;
template <> struct FftPlan<64> { static constexpr int T = 8; using R = Radices<8, 8>; };
template <> struct FftPlan<128> { static constexpr int T = 8; using R = Radices<16, 8>; };
template <> struct FftPlan<256> { static constexpr int T = 16; using R = Radices<16, 16>; };
template <> struct FftPlan<512> { static constexpr int T = 32; using R = Radices<16, 8, 4>; };
template <> struct FftPlan<1024> { static constexpr int T = 64; using R = Radices<16, 16, 4>; };
template <> struct FftPlan<2048> { static constexpr int T = 64; using R = Radices<16, 16, 8>; };
template <> struct FftPlan<4096> { static constexpr int T = 128; using R = Radices<16, 16, 16>; };
template <> struct FftPlan<96> { static constexpr int T = 8; using R = Radices<4, 2, 12>; };
template <> struct FftPlan<160> { static constexpr int T = 8; using R = Radices<4, 4, 10>; };
template <> struct FftPlan<192> { static constexpr int T = 16; using R = Radices<4, 4, 12>; };
template <> struct FftPlan<320> { static constexpr int T = 16; using R = Radices<4, 4, 20>; };
template <> struct FftPlan<384> { static constexpr int T = 16; using R = Radices<4, 8, 12>; };
template <> struct FftPlan<640> { static constexpr int T = 32; using R = Radices<4, 4, 4, 10>; };
template <> struct FftPlan<768> { static constexpr int T = 32; using R = Radices<8, 8, 12>; };
template <> struct FftPlan<1280> { static constexpr int T = 64; using R = Radices<4, 4, 4, 20>; };
template <> struct FftPlan<1536> { static constexpr int T = 64; using R = Radices<2, 8, 8, 12>; };
template <> struct FftPlan<2560> { static constexpr int T = 64; using R = Radices<8, 8, 4, 10>; };
template <> struct FftPlan<3072> { static constexpr int T = 64; using R = Radices<16, 16, 12>; };

// LDS index with one pad slot every 32 complex values, and 4 more slots
// between the regions of neighbouring transforms: breaks the power-of-two
// strides of the Stockham scatter across 64 four-byte banks.
// LDS padding of exchange p (the writes of pass p and the reads of pass
// p + 1): element x lives at x + M_p (x >> 5).  The multipliers are chosen per
// plan (bank model: 64 banks of 4 B, 32 lanes per cycle, 8-byte elements) so
// that both access patterns of every exchange avoid bank conflicts; any M_p
// keeps the padded addresses affine in the element index, because every write
// stride is a power of two.
template <int... Ms>
struct PadMults {};
template <int L>
struct PadPlan {
  using M = PadMults<>;  // all 1
};
template <> struct PadPlan<512> { using M = PadMults<1, 4>; };
template <> struct PadPlan<640> { using M = PadMults<1, 4, 8>; };
template <> struct PadPlan<768> { using M = PadMults<1, 4>; };
template <> struct PadPlan<1024> { using M = PadMults<1, 2>; };
template <> struct PadPlan<1280> { using M = PadMults<1, 4, 8>; };
template <> struct PadPlan<1536> { using M = PadMults<1, 2, 4>; };
template <> struct PadPlan<2048> { using M = PadMults<1, 2>; };
template <> struct PadPlan<2560> { using M = PadMults<1, 4, 0>; };
template <> struct PadPlan<3072> { using M = PadMults<1, 2>; };
template <> struct PadPlan<4096> { using M = PadMults<1, 2>; };

template <int P, typename Pack>
struct PadAt {
  static constexpr int value = 1;
};
template <int P, int M0, int... Ms>
struct PadAt<P, PadMults<M0, Ms...>> {
  static constexpr int value = P == 0 ? M0 : PadAt<P - 1, PadMults<Ms...>>::value;
};
template <int... Ms>
constexpr int pad_max(PadMults<Ms...>) {
  int m = 1;
  for (int x : {1, Ms...}) m = x > m ? x : m;
  return m;
}

template <int M>
__device__ __forceinline__ int lpad(int i) { return i + M * (i >> 5); }
constexpr int lpad_c(int i, int M) { return i + M * (i >> 5); }

// Exchange addressing.  Output r of butterfly mb of lane t in a pass of radix
// R after radices multiplying to S goes to position wpos(t, mb, r); lane t
// reads back positions t + T*i.  For every plan here the padded address of
// each (mb, r), and of each i, is the lane's own (0, 0) (or i = 0) address
// plus an offset that is the same for all lanes (checked at compile time
// below), so an exchange costs one per-lane base and immediate LDS offsets
// rather than an address computation per value.
template <int T, int R, int S>
constexpr int wpos(int t, int mb, int r) {
  return ((t + T * mb) / S) * S * R + (t + T * mb) % S + r * S;
}
template <int T, int R, int S, int NB, int M>
constexpr bool lane_uniform_writes() {
  for (int t = 0; t < T; ++t)
    for (int mb = 0; mb < NB; ++mb)
      for (int r = 0; r < R; ++r)
        if (lpad_c(wpos<T, R, S>(t, mb, r), M) - lpad_c(wpos<T, R, S>(t, 0, 0), M) !=
            lpad_c(wpos<T, R, S>(0, mb, r), M) - lpad_c(wpos<T, R, S>(0, 0, 0), M))
          return false;
  return true;
}
template <int T, int E, int M>
constexpr bool lane_uniform_reads() {
  for (int t = 0; t < T; ++t)
    for (int i = 0; i < E; ++i)
      if (lpad_c(t + T * i, M) - lpad_c(t, M) != lpad_c(T * i, M)) return false;
  return true;
}
template <int T, int R, int S, int M>
constexpr int woff(int mb, int r) {
  return lpad_c(wpos<T, R, S>(0, mb, r), M) - lpad_c(wpos<T, R, S>(0, 0, 0), M);
}
template <int L>
constexpr int lds_len() { return L + pad_max(typename PadPlan<L>::M{}) * (L / 32) + 4; }

// Half-width exchange: the real parts of a transform cross the LDS first,
// then the imaginary parts, through one region of four-byte slots, which
// halves the LDS a transform holds (and so raises the occupancy of the
// LDS-bound row passes) for twice the LDS instructions.  The exchanges are
// ordered by the same waits as the complex ones (within a wavefront up to 64
// threads, block barriers beyond).  Row stride (in four-byte slots
// beyond the padded length) and per-exchange padding come from a bank model
// of four-byte accesses (64 banks, 32 or 64 lanes a cycle), under which
// the exchanges of the plans of at most 32 threads are free of conflicts.
template <int L>
struct HalfPlan {
  static constexpr bool ok = false;
  static constexpr int extra = 0;
  using M = PadMults<>;
};
template <> struct HalfPlan<64> { static constexpr bool ok = true; static constexpr int extra = 5; using M = PadMults<0>; };
template <> struct HalfPlan<96> { static constexpr bool ok = true; static constexpr int extra = 3; using M = PadMults<0, 0>; };
template <> struct HalfPlan<128> { static constexpr bool ok = true; static constexpr int extra = 4; using M = PadMults<1>; };
template <> struct HalfPlan<160> { static constexpr bool ok = true; static constexpr int extra = 3; using M = PadMults<0, 0>; };
template <> struct HalfPlan<192> { static constexpr bool ok = true; static constexpr int extra = 24; using M = PadMults<1, 4>; };
template <> struct HalfPlan<256> { static constexpr bool ok = true; static constexpr int extra = 8; using M = PadMults<1>; };
template <> struct HalfPlan<320> { static constexpr bool ok = true; static constexpr int extra = 8; using M = PadMults<1, 4>; };
template <> struct HalfPlan<384> { static constexpr bool ok = true; static constexpr int extra = 0; using M = PadMults<1, 4>; };
template <> struct HalfPlan<512> { static constexpr bool ok = true; static constexpr int extra = 32; using M = PadMults<1, 4>; };
template <> struct HalfPlan<640> { static constexpr bool ok = true; static constexpr int extra = 0; using M = PadMults<1, 4, 8>; };
template <> struct HalfPlan<768> { static constexpr bool ok = true; static constexpr int extra = 0; using M = PadMults<1, 4>; };
// one transform per wavefront (the row stride does not matter): these keep
// some two-way conflicts under the 64-lane model (none beyond the two-cycle
// minimum under the 32-lane one).  Which passes use a plan is decided per
// pass by the kernels.
template <> struct HalfPlan<1024> { static constexpr bool ok = true; static constexpr int extra = 0; using M = PadMults<1, 2>; };
template <> struct HalfPlan<1280> { static constexpr bool ok = true; static constexpr int extra = 0; using M = PadMults<1, 1, 8>; };
template <> struct HalfPlan<1536> { static constexpr bool ok = true; static constexpr int extra = 0; using M = PadMults<0, 1, 4>; };
template <> struct HalfPlan<2048> { static constexpr bool ok = true; static constexpr int extra = 0; using M = PadMults<1, 2>; };
template <> struct HalfPlan<2560> { static constexpr bool ok = true; static constexpr int extra = 0; using M = PadMults<1, 4, 0>; };
template <> struct HalfPlan<3072> { static constexpr bool ok = true; static constexpr int extra = 0; using M = PadMults<1, 2>; };
// two wavefronts per transform (block barriers); two-way conflicts remain in
// the first exchange under the 64-lane model
template <> struct HalfPlan<4096> { static constexpr bool ok = true; static constexpr int extra = 0; using M = PadMults<1, 2>; };
// four-byte slots of one transform's region
template <int L>
constexpr int lds_len_half() { return L + pad_max(typename HalfPlan<L>::M{}) * (L / 32) + HalfPlan<L>::extra; }

// Twiddle table layout.  Pass p (radix R after radices multiplying to S > 1)
// owns S * tw_per(R, S) consecutive entries; a butterfly reads its twiddles
// from one base address.  Radix 4: entries [k][0] = (cos a, tan a) and
// [k][1] = (cos 2a, tan 2a), a = -2 pi k / (4 S) (the form of dft4_tw below);
// other radices: entry [k][r - 1] = exp(-2 pi i k r / (S R)).
constexpr int tw_per(int R, int S) { return S > 1 ? (R == 4 ? 2 : R - 1) : 0; }
template <int S, int... Rs>
struct TwSize;
template <int S>
struct TwSize<S> {
  static constexpr int value = 0;
};
template <int S, int R, int... Rest>
struct TwSize<S, R, Rest...> {
  static constexpr int value = S * tw_per(R, S) + TwSize<S * R, Rest...>::value;
};
template <int L, typename Rad>
struct TwTable;
template <int L, int... Rs>
struct TwTable<L, Radices<Rs...>> {
  static constexpr int size = TwSize<1, Rs...>::value;
};
template <int L>
constexpr int twiddle_table_size() { return TwTable<L, typename FftPlan<L>::R>::size; }

// Ordering of the LDS exchange between passes.  A transform whose T threads
// lie inside one wavefront only needs its own LDS writes to have landed
// before its reads (DS instructions of a wavefront complete in order; the
// explicit wait and the memory clobber also stop the compiler from moving
// the reads above the writes).  Wider transforms synchronise the block.
template <int T>
__device__ __forceinline__ void xsync() {
  if constexpr (T <= 64) {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  } else {
    __syncthreads();
  }
}

// Hides the twiddle-table pointer from loop-invariant code motion, so the
// table loads of a transform inside a loop are issued per transform instead
// of being hoisted into (and holding) registers for the whole loop.
__device__ __forceinline__ const cf *opaque(const cf *p) {
  int zero = 0;
  asm volatile("" : "+s"(zero));
  return p + zero;
}

// Same for a per-lane index: the LDS and table addresses derived from it are
// then recomputed inside each transform rather than kept live across a loop.
__device__ __forceinline__ int opaque_lane(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Radix-4 butterfly of a Stockham pass with its input twiddles w, w^2, w^3
// (inputs u[r] scaled by w^r, then the 4-point DFT), factored as in Linzer
// and Feig's FFT for fused multiply-add units: w^2 on the pairs (u0, u2) and
// (u1, u3), then w on the odd half, each product written c (x - t y, y + t x)
// with the cosine c folded into the butterfly's fused multiply-adds.  24 FMAs
// against 12 for three complex products plus 16 additions.  w1 = (cos a,
// tan a), w2 = (cos 2a, tan 2a), the tangents already signed for DIR; the
// table clamps |cos| to at least 2^-26, where the represented twiddle is
// off by less than half an FP32 ulp of 1.
template <int DIR>
__device__ __forceinline__ void dft4_tw(cf *u, cf w1, cf w2) {
  const float p2x = fmaf(-w2.y, u[2].y, u[2].x), p2y = fmaf(w2.y, u[2].x, u[2].y);
  const float p3x = fmaf(-w2.y, u[3].y, u[3].x), p3y = fmaf(w2.y, u[3].x, u[3].y);
  const cf a = cmake(fmaf(w2.x, p2x, u[0].x), fmaf(w2.x, p2y, u[0].y));
  const cf b = cmake(fmaf(-w2.x, p2x, u[0].x), fmaf(-w2.x, p2y, u[0].y));
  const cf e = cmake(fmaf(w2.x, p3x, u[1].x), fmaf(w2.x, p3y, u[1].y));
  const cf f = cmake(fmaf(-w2.x, p3x, u[1].x), fmaf(-w2.x, p3y, u[1].y));
  const float ex = fmaf(-w1.y, e.y, e.x), ey = fmaf(w1.y, e.x, e.y);
  const float fx = fmaf(-w1.y, f.y, f.x), fy = fmaf(w1.y, f.x, f.y);
  u[0] = cmake(fmaf(w1.x, ex, a.x), fmaf(w1.x, ey, a.y));
  u[2] = cmake(fmaf(-w1.x, ex, a.x), fmaf(-w1.x, ey, a.y));
  // DIR i w f = DIR (-c fy, c fx)
  constexpr float sg = DIR > 0 ? 1.f : -1.f;
  u[1] = cmake(fmaf(-sg * w1.x, fy, b.x), fmaf(sg * w1.x, fx, b.y));
  u[3] = cmake(fmaf(sg * w1.x, fy, b.x), fmaf(-sg * w1.x, fx, b.y));
}

// Input twiddles of butterfly j of a pass (radix R after radices multiplying
// to S, its table entries from OFF), then its R-point DFT, in place.
template <int R, int S, int OFF, int DIR>
__device__ __forceinline__ void twiddled_dft(cf (&u)[R], const cf *__restrict__ twp, int j) {
  if constexpr (S > 1 && R == 4) {
    const cf *tb = twp + OFF + (j % S) * 2;
    cf w1 = tb[0], w2 = tb[1];
    if constexpr (DIR > 0) {
      w1.y = -w1.y;
      w2.y = -w2.y;
    }
    dft4_tw<DIR>(u, w1, w2);
  } else {
    if constexpr (S > 1) {
      const cf *tb = twp + OFF + (j % S) * (R - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cf w = tb[r - 1];
        if constexpr (DIR > 0) w.y = -w.y;
        u[r] = cmul(u[r], w);
      }
    }
    Dft<R, DIR>::run(u);
  }
}

// One Stockham pass of radix R after passes whose radices multiply to S;
// its twiddles start at entry OFF of the table; its exchange pads by M.
template <int L, int T, int DIR, int R, int S, int OFF, bool LAST, int M>
__device__ __forceinline__ void stockham_pass(cf (&v)[L / T], cf *__restrict__ buf, int t,
                                              const cf *__restrict__ tw) {
  constexpr int E = L / T;
  constexpr int NB = E / R;
  static_assert(E % R == 0, "radix must divide the per-thread count");
  const cf *twp = opaque(tw);
#pragma unroll
  for (int mb = 0; mb < NB; ++mb) {
    const int j = t + T * mb;
    cf u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[mb + r * NB];
    twiddled_dft<R, S, OFF, DIR>(u, twp, j);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[mb + r * NB] = u[r];
    } else if constexpr (lane_uniform_writes<T, R, S, NB, M>()) {
      cf *wb = buf + lpad<M>(wpos<T, R, S>(t, 0, 0));
#pragma unroll
      for (int r = 0; r < R; ++r) wb[woff<T, R, S, M>(mb, r)] = u[r];
    } else {
      const int base = (j / S) * S * R + (j % S);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lpad<M>(base + r * S)] = u[r];
    }
  }
  if constexpr (!LAST) {
    xsync<T>();
    if constexpr (lane_uniform_reads<T, E, M>()) {
      const cf *rb = buf + lpad<M>(t);
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = rb[lpad_c(T * i, M)];
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = buf[lpad<M>(t + T * i)];
    }
    xsync<T>();
  }
}

// The same pass with the half-width exchange (see HalfPlan): butterflies in
// place, then the real parts and the imaginary parts cross the LDS in turn.
template <int L, int T, int DIR, int R, int S, int OFF, bool LAST, int M>
__device__ __forceinline__ void stockham_pass_half(cf (&v)[L / T], float *__restrict__ buf, int t,
                                                   const cf *__restrict__ tw) {
  constexpr int E = L / T;
  constexpr int NB = E / R;
  static_assert(E % R == 0, "radix must divide the per-thread count");
  const cf *twp = opaque(tw);
#pragma unroll
  for (int mb = 0; mb < NB; ++mb) {
    const int j = t + T * mb;
    cf u[R];
#pragma unroll
    for (int r = 0; r < R; ++r) u[r] = v[mb + r * NB];
    twiddled_dft<R, S, OFF, DIR>(u, twp, j);
#pragma unroll
    for (int r = 0; r < R; ++r) v[mb + r * NB] = u[r];
  }
  if constexpr (!LAST) {
    static_assert(lane_uniform_writes<T, R, S, NB, M>() && lane_uniform_reads<T, E, M>(),
                  "half-width exchange plans use lane-uniform offsets");
    float *wb = buf + lpad<M>(wpos<T, R, S>(t, 0, 0));
    const float *rb = buf + lpad<M>(t);
#pragma unroll
    for (int mb = 0; mb < NB; ++mb)
#pragma unroll
      for (int r = 0; r < R; ++r) wb[woff<T, R, S, M>(mb, r)] = v[mb + r * NB].x;
    xsync<T>();
#pragma unroll
    for (int i = 0; i < E; ++i) v[i].x = rb[lpad_c(T * i, M)];
    xsync<T>();
#pragma unroll
    for (int mb = 0; mb < NB; ++mb)
#pragma unroll
      for (int r = 0; r < R; ++r) wb[woff<T, R, S, M>(mb, r)] = v[mb + r * NB].y;
    xsync<T>();
#pragma unroll
    for (int i = 0; i < E; ++i) v[i].y = rb[lpad_c(T * i, M)];
    xsync<T>();
  }
}

template <int L, int T, int DIR, int S, int OFF, int P, int R, int... Rest>
__device__ __forceinline__ void run_passes_half(cf (&v)[L / T], float *buf, int t, const cf *tw) {
  stockham_pass_half<L, T, DIR, R, S, OFF, sizeof...(Rest) == 0, PadAt<P, typename HalfPlan<L>::M>::value>(
      v, buf, t, tw);
  if constexpr (sizeof...(Rest) > 0)
    run_passes_half<L, T, DIR, S * R, OFF + S * tw_per(R, S), P + 1, Rest...>(v, buf, t, tw);
}

template <int L, int DIR, int... Rs>
__device__ __forceinline__ void fft_half_impl(cf (&v)[L / FftPlan<L>::T], float *buf, int t, const cf *tw,
                                              Radices<Rs...>) {
  run_passes_half<L, FftPlan<L>::T, DIR, 1, 0, 0, Rs...>(v, buf, t, tw);
}

template <int L, int T, int DIR, int S, int OFF, int P, int R, int... Rest>
__device__ __forceinline__ void run_passes(cf (&v)[L / T], cf *buf, int t, const cf *tw) {
  stockham_pass<L, T, DIR, R, S, OFF, sizeof...(Rest) == 0, PadAt<P, typename PadPlan<L>::M>::value>(v, buf, t,
                                                                                                     tw);
  if constexpr (sizeof...(Rest) > 0)
    run_passes<L, T, DIR, S * R, OFF + S * tw_per(R, S), P + 1, Rest...>(v, buf, t, tw);
}

template <int L, int DIR, int... Rs>
__device__ __forceinline__ void fft_impl(cf (&v)[L / FftPlan<L>::T], cf *buf, int t, const cf *tw,
                                         Radices<Rs...>) {
  run_passes<L, FftPlan<L>::T, DIR, 1, 0, 0, Rs...>(v, buf, t, tw);
}

// Host: fills the table of FftPlan<L> (FP64 angles, rounded once to FP32).
template <int S, int... Rs>
struct TwFill;
template <int S>
struct TwFill<S> {
  static void run(float2 *, int) {}
};
template <int S, int R, int... Rest>
struct TwFill<S, R, Rest...> {
  static void run(float2 *out, int off) {
    if (S > 1 && R == 4) {
      for (int k = 0; k < S; ++k)
        for (int m = 1; m <= 2; ++m) {
          const double a = -2.0 * 3.14159265358979323846 * double(k) * double(m) / double(S * R);
          double c = __builtin_cos(a);
          if (__builtin_fabs(c) < 0x1p-26) c = 0x1p-26;
          out[off + k * 2 + (m - 1)] = make_float2(float(c), float(__builtin_sin(a) / c));
        }
    } else if (S > 1) {
      for (int k = 0; k < S; ++k)
        for (int r = 1; r < R; ++r) {
          const double a = -2.0 * 3.14159265358979323846 * double(k) * double(r) / double(S * R);
          out[off + k * (R - 1) + (r - 1)] = make_float2(float(__builtin_cos(a)), float(__builtin_sin(a)));
        }
    }
    TwFill<S * R, Rest...>::run(out, off + S * tw_per(R, S));
  }
};
template <int L, int... Rs>
void fill_twiddles_impl(float2 *out, Radices<Rs...>) {
  TwFill<1, Rs...>::run(out, 0);
}
template <int L>
void fill_twiddles(float2 *out) {
  fill_twiddles_impl<L>(out, typename FftPlan<L>::R{});
}

// In-register FFT of length L (DIR = -1 forward, +1 inverse, unnormalised).
// buf: this transform's private LDS region of lds_len<L>() complex values.
// Transforms of at most 64 threads synchronise only their own wavefront, so
// every thread of a wavefront must call it together (uniform control flow);
// wider ones use block barriers and need the whole block.
template <int L, int DIR>
__device__ __forceinline__ void fft(cf (&v)[L / FftPlan<L>::T], cf *buf, int t, const cf *tw) {
  // the mask restores the known range 0 <= t < T after the opaque copy, so
  // padded LDS addresses of t + T*i fold into immediate offsets
  fft_impl<L, DIR>(v, buf, opaque_lane(t) & (FftPlan<L>::T - 1), tw, typename FftPlan<L>::R{});
}

// Same transform with the half-width exchange; buf: lds_len_half<L>() floats.
template <int L, int DIR>
__device__ __forceinline__ void fft_half(cf (&v)[L / FftPlan<L>::T], float *buf, int t, const cf *tw) {
  static_assert(HalfPlan<L>::ok, "no half-width exchange plan for this length");
  fft_half_impl<L, DIR>(v, buf, opaque_lane(t) & (FftPlan<L>::T - 1), tw, typename FftPlan<L>::R{});
}

}  // namespace dev
}  // namespace litho
