// Mixed-radix complex FFT on LDS-staged pencils for gfx950.
//
// A workgroup holds W pencils of length L in LDS as buf[i * W + p] (pencil p fastest, so a
// 64-lane wave touching consecutive p hits consecutive banks).  Each radix stage is an
// in-place Stockham autosort step: every thread loads the R inputs of its butterflies
// into registers, the group synchronises, then applies twiddles, the radix-R DFT and
// writes the R outputs to their self-sorted places.  Stages follow a runtime plan
// (radices and running products), so one kernel instance serves every supported length.
//
// Forward transforms use exp(-2 pi i j k / L); inverse ones use the conjugate and are
// unnormalised (the caller folds 1/L into its data).
//
// Every routine is generic in the complex type V: float2 (the correlation of the product
// fields) or double2 (the exact overlap counts of a general fixed-side mask, whose FP64
// transform error stays far below the 1/2 that rounding to an integer tolerates).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace csngf {

constexpr int kMaxStages = 12;
constexpr int kMaxLen = 512;

struct FftPlan {
  int L;                    // transform length
  int nst;                  // number of stages
  int radix[kMaxStages];    // radix of each stage
  int ns[kMaxStages];       // product of the radices of all earlier stages
  int tw_off;               // offset of this length's table W_L^j, j < L, in the table buffer
};

// scalar type of a complex vector type, and construction
template <typename V>
using scalar_t = std::remove_reference_t<decltype(V{}.x)>;
template <typename V>
__device__ __forceinline__ V cplx(scalar_t<V> x, scalar_t<V> y) {
  V r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename V>
__device__ __forceinline__ V czero() {
  return cplx<V>(scalar_t<V>(0), scalar_t<V>(0));
}
__device__ __forceinline__ float fmadd(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return fma(a, b, c); }

template <typename V>
__device__ __forceinline__ V cadd(V a, V b) { return cplx<V>(a.x + b.x, a.y + b.y); }
template <typename V>
__device__ __forceinline__ V csub(V a, V b) { return cplx<V>(a.x - b.x, a.y - b.y); }
template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
  return cplx<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename V>
__device__ __forceinline__ V rot_i(V a) {
  return INV ? cplx<V>(-a.y, a.x) : cplx<V>(a.y, -a.x);
}

// ---------------------------------------------------------------- small DFTs
// NZ: inputs x[m] with m >= NZ are known to be zero (the first stage of a zero-padded
// transform), so the sums and differences that involve them are skipped.
template <int NZ, int M, typename V>
__device__ __forceinline__ V add_nz(const V* x, int a) {  // x[a] + x[M] with x[M] maybe zero
  return M >= NZ ? x[a] : cadd(x[a], x[M]);
}
template <int NZ, int M, typename V>
__device__ __forceinline__ V sub_nz(const V* x, int a) {  // x[a] - x[M] with x[M] maybe zero
  return M >= NZ ? x[a] : csub(x[a], x[M]);
}

template <bool INV, int NZ = 2, typename V>
__device__ __forceinline__ void dft2(V* x) {
  V a = x[0];
  x[0] = add_nz<NZ, 1>(x, 0);
  x[1] = NZ > 1 ? csub(a, x[1]) : a;
}

template <bool INV, int NZ = 4, typename V>
__device__ __forceinline__ void dft4(V* x) {
  V t0 = add_nz<NZ, 2>(x, 0), t1 = sub_nz<NZ, 2>(x, 0);
  V t2, t3;
  if constexpr (NZ > 1) {
    t2 = add_nz<NZ, 3>(x, 1);
    t3 = rot_i<INV>(sub_nz<NZ, 3>(x, 1));
  } else {
    t2 = t3 = czero<V>();
  }
  x[0] = cadd(t0, t2);
  x[2] = csub(t0, t2);
  x[1] = cadd(t1, t3);
  x[3] = csub(t1, t3);
}

template <bool INV, int NZ = 8, typename V>
__device__ __forceinline__ void dft8(V* x) {
  static_assert(NZ >= 4, "dft8 prunes at most its upper half");
  using S = scalar_t<V>;
  constexpr S h = std::is_same<S, float>::value ? S(0.70710678118654752f) : S(0.70710678118654752440);
  V a[4], b[4];
  a[0] = add_nz<NZ, 4>(x, 0); b[0] = sub_nz<NZ, 4>(x, 0);
  a[1] = add_nz<NZ, 5>(x, 1); b[1] = sub_nz<NZ, 5>(x, 1);
  a[2] = add_nz<NZ, 6>(x, 2); b[2] = sub_nz<NZ, 6>(x, 2);
  a[3] = add_nz<NZ, 7>(x, 3); b[3] = sub_nz<NZ, 7>(x, 3);
  // b[k] *= W8^k  (W8 = exp(-i pi/4) forward, conjugate inverse)
  b[1] = INV ? cplx<V>(h * (b[1].x - b[1].y), h * (b[1].x + b[1].y))
             : cplx<V>(h * (b[1].x + b[1].y), h * (b[1].y - b[1].x));
  b[2] = rot_i<INV>(b[2]);
  b[3] = INV ? cplx<V>(-h * (b[3].x + b[3].y), h * (b[3].x - b[3].y))
             : cplx<V>(h * (b[3].y - b[3].x), -h * (b[3].x + b[3].y));
  dft4<INV>(a);
  dft4<INV>(b);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    x[2 * m] = a[m];
    x[2 * m + 1] = b[m];
  }
}

// cos(2 pi j / R) and sin(2 pi j / R) for j = 1 .. (R-1)/2
template <int R> struct OddRoots;
template <> struct OddRoots<3> {
  static constexpr float c[1] = {-0.5f};
  static constexpr float s[1] = {0.86602540378443871f};
};
template <> struct OddRoots<5> {
  static constexpr float c[2] = {0.30901699437494745f, -0.80901699437494734f};
  static constexpr float s[2] = {0.95105651629515353f, 0.58778525229247325f};
};
template <> struct OddRoots<7> {
  static constexpr float c[3] = {0.62348980185873359f, -0.22252093395631434f, -0.90096886790241903f};
  static constexpr float s[3] = {0.7818314824680298f, 0.97492791218182362f, 0.43388373911755823f};
};
template <> struct OddRoots<11> {
  static constexpr float c[5] = {0.84125353283118121f, 0.41541501300188644f, -0.142314838273285f,
                                 -0.65486073394528499f, -0.95949297361449737f};
  static constexpr float s[5] = {0.54064081745559756f, 0.90963199535451833f, 0.9898214418809328f,
                                 0.75574957435425827f, 0.28173255684142967f};
};
// the same in double precision
template <int R> struct OddRootsD;
template <> struct OddRootsD<3> {
  static constexpr double c[1] = {-0.5};
  static constexpr double s[1] = {0.86602540378443864676};
};
template <> struct OddRootsD<5> {
  static constexpr double c[2] = {0.30901699437494742410, -0.80901699437494742410};
  static constexpr double s[2] = {0.95105651629515357212, 0.58778525229247312917};
};
template <> struct OddRootsD<7> {
  static constexpr double c[3] = {0.62348980185873353053, -0.22252093395631440429, -0.90096886790241912624};
  static constexpr double s[3] = {0.78183148246802980871, 0.97492791218182360702, 0.43388373911755812048};
};
template <> struct OddRootsD<11> {
  static constexpr double c[5] = {0.84125353283118116886, 0.41541501300188642553, -0.14231483827328514044,
                                  -0.65486073394528506406, -0.95949297361449738989};
  static constexpr double s[5] = {0.54064081745559758211, 0.90963199535451837141, 0.98982144188093273238,
                                  0.75574957435425828377, 0.28173255684142969771};
};
template <typename S, int R>
__device__ __forceinline__ S root_c(int i) {
  if constexpr (std::is_same<S, float>::value) return OddRoots<R>::c[i];
  else return OddRootsD<R>::c[i];
}
template <typename S, int R>
__device__ __forceinline__ S root_s(int i) {
  if constexpr (std::is_same<S, float>::value) return OddRoots<R>::s[i];
  else return OddRootsD<R>::s[i];
}

// Odd prime R: pair x_m with x_{R-m}; y_k = A_k -+ i B_k, y_{R-k} = A_k +- i B_k with
// A_k = x_0 + sum_m (x_m + x_{R-m}) cos(2 pi k m / R), B_k = sum_m (x_m - x_{R-m}) sin(..).
template <int R, bool INV, int NZ = R, typename V>
__device__ __forceinline__ void dft_odd(V* x) {
  using S = scalar_t<V>;
  constexpr int h = (R - 1) / 2;
  static_assert(NZ > h, "dft_odd prunes at most its upper half");
  V a[h + 1], b[h + 1];
  V y0 = x[0];
#pragma unroll
  for (int m = 1; m <= h; ++m) {
    const bool upper_zero = R - m >= NZ;   // compile time after unrolling
    a[m] = upper_zero ? x[m] : cadd(x[m], x[R - m]);
    b[m] = upper_zero ? x[m] : csub(x[m], x[R - m]);
    y0 = cadd(y0, a[m]);
  }
  V out[R];
  out[0] = y0;
#pragma unroll
  for (int k = 1; k <= h; ++k) {
    V A = x[0];
    V B = czero<V>();
#pragma unroll
    for (int m = 1; m <= h; ++m) {
      const int j = (k * m) % R;
      const S c = (j <= h) ? root_c<S, R>(j - 1) : root_c<S, R>(R - j - 1);
      const S s = (j <= h) ? root_s<S, R>(j - 1) : -root_s<S, R>(R - j - 1);
      A.x = fmadd(a[m].x, c, A.x);
      A.y = fmadd(a[m].y, c, A.y);
      B.x = fmadd(b[m].x, s, B.x);
      B.y = fmadd(b[m].y, s, B.y);
    }
    if (!INV) {
      out[k] = cplx<V>(A.x + B.y, A.y - B.x);
      out[R - k] = cplx<V>(A.x - B.y, A.y + B.x);
    } else {
      out[k] = cplx<V>(A.x - B.y, A.y + B.x);
      out[R - k] = cplx<V>(A.x + B.y, A.y - B.x);
    }
  }
#pragma unroll
  for (int k = 0; k < R; ++k) x[k] = out[k];
}

template <int R, bool INV, int NZ = R, typename V>
__device__ __forceinline__ void dft(V* x) {
  if constexpr (R == 2) dft2<INV, NZ>(x);
  else if constexpr (R == 4) dft4<INV, NZ>(x);
  else if constexpr (R == 8) dft8<INV, NZ>(x);
  else dft_odd<R, INV, NZ>(x);
}

// ---------------------------------------------------------------- one Stockham stage
// LW is the largest L * W this instance must handle; it bounds the butterflies per thread.
template <int R, int W, int T, int LW, bool INV, typename V>
__device__ __forceinline__ void fft_stage(V* __restrict__ buf, const V* __restrict__ tw,
                                          int L, int ns) {
  constexpr int NB = (LW / R + T - 1) / T;
  const int lr = L / R;
  const int nbf = lr * W;
  const int twstep = L / (ns * R);
  V v[NB][R];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int bf = (int)threadIdx.x + u * T;
    if (bf < nbf) {
      const int p = bf % W, j = bf / W;
#pragma unroll
      for (int t = 0; t < R; ++t) v[u][t] = buf[(j + t * lr) * W + p];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int bf = (int)threadIdx.x + u * T;
    if (bf < nbf) {
      const int p = bf % W, j = bf / W;
      const int k = j % ns, q = j / ns;
      if (ns > 1) {
#pragma unroll
        for (int t = 1; t < R; ++t) {
          V w = tw[t * k * twstep];
          if (INV) w.y = -w.y;
          v[u][t] = cmul(v[u][t], w);
        }
      }
      dft<R, INV>(v[u]);
      const int base = q * ns * R + k;
#pragma unroll
      for (int t = 0; t < R; ++t) buf[(base + t * ns) * W + p] = v[u][t];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- 24-bit index arithmetic
// Full-rate 24-bit integer multiplies (operands < 2^24).  Written as instructions: the
// compiler turns __umul24 into a general 32-bit multiply, a quarter-rate instruction,
// wherever it can prove the operands small but loses that fact before choosing the
// instruction.
// a * C for a compile-time C (a literal operand; powers of two are shifts)
template <unsigned C>
__device__ __forceinline__ unsigned mul24c(unsigned a) {
  static_assert(C < (1u << 24), "24-bit constant");
  if constexpr ((C & (C - 1)) == 0) {
    return a * C;
  } else {
    unsigned r;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "i"(C), "v"(a));
    return r;
  }
}
// a * b + c with a workgroup-uniform b (held in a scalar register)
__device__ __forceinline__ unsigned mad24u(unsigned a, unsigned b, unsigned c) {
  unsigned r;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
  return r;
}

// ---------------------------------------------------------------- compile-time plans
// floor(j / D) for 0 <= j < MAXJ with one full-rate 24-bit multiply and a shift instead of
// the quarter-rate 32-bit multiplies of a general division: with M = ceil(2^S / D) and
// e = M D - 2^S < D, j M / 2^S = j / D + j e / (D 2^S), and j e < 2^S keeps the floor exact.
template <unsigned D, unsigned MAXJ>
__device__ __forceinline__ unsigned div_small(unsigned j) {
  if constexpr ((D & (D - 1)) == 0) {
    return j / D;
  } else {
    constexpr unsigned S = 20;
    constexpr unsigned long long M = ((1ull << S) + D - 1) / D;
    static_assert((unsigned long long)(MAXJ - 1) * (M * D - (1ull << S)) < (1ull << S), "inexact");
    static_assert(M < (1u << 24) && (unsigned long long)(MAXJ - 1) * M < (1ull << 32), "24-bit range");
    return mul24c<(unsigned)M>(j) >> S;
  }
}

struct CPlan {
  int nst;
  int r[kMaxStages];
  int ns[kMaxStages];
};

// Same factorisation as the host plan: odd radices first (11, 7, 5, 3), then 8, 4, 2.
constexpr CPlan make_cplan(int L) {
  CPlan p{0, {0}, {0}};
  int n = L;
  const int odd[4] = {11, 7, 5, 3};
  for (int i = 0; i < 4; ++i)
    while (n % odd[i] == 0) { p.r[p.nst++] = odd[i]; n /= odd[i]; }
  while (n % 8 == 0) { p.r[p.nst++] = 8; n /= 8; }
  while (n % 4 == 0) { p.r[p.nst++] = 4; n /= 4; }
  while (n % 2 == 0) { p.r[p.nst++] = 2; n /= 2; }
  int ns = 1;
  for (int s = 0; s < p.nst; ++s) { p.ns[s] = ns; ns *= p.r[s]; }
  return p;
}

// Twiddles of a compile-time plan, stored by stage so that the R - 1 factors of a butterfly
// are adjacent (one address per butterfly, the factors at constant offsets): stage s >= 1,
// with radix R and stride NS, holds w^(t k L / (NS R)) for k = 0 .. NS - 1, t = 1 .. R - 1
// at NS - R_0 + k (R - 1) + t - 1, where R_0 is the first stage's radix.  (Stage 0 has
// NS = 1, so k = 0 and no factors; the earlier stages' blocks NS_s (R_s - 1) sum to
// NS - R_0.)  The whole table has L - R_0 entries, fewer than the plain table's L.
template <int L, int NS>
constexpr int staged_tw_first() {
  return NS - make_cplan(L).r[0];
}
template <int L>
constexpr int staged_tw_size() {
  return L - make_cplan(L).r[0];
}
// index into the plain table (w^i at i) of staged entry e, for the stages S, S + 1, ...
template <int L, int S>
__device__ __forceinline__ unsigned staged_tw_source(unsigned e) {
  constexpr CPlan P = make_cplan(L);
  if constexpr (S >= P.nst) {
    return 0;
  } else {
    constexpr int R = P.r[S], NS = P.ns[S];
    constexpr unsigned end = (unsigned)(NS * R - P.r[0]);
    if (e < end) {
      const unsigned d = e - (unsigned)staged_tw_first<L, NS>();
      const unsigned k = div_small<R - 1, NS * (R - 1)>(d), t = d - k * (R - 1) + 1;
      return t * k * (unsigned)(L / (NS * R));
    }
    return staged_tw_source<L, S + 1>(e);
  }
}

// Whole transform on the run-time plan pl (any supported length up to kMaxLen) with the
// plain twiddle table.  Caller has synchronised after filling buf; on return buf holds the
// result in natural order and the group is synchronised.
template <int W, int T, bool INV, typename V>
__device__ void fft_lds(V* __restrict__ buf, const V* __restrict__ tw, const FftPlan& pl) {
  constexpr int LW = kMaxLen * W;
  for (int s = 0; s < pl.nst; ++s) {
    const int ns = pl.ns[s];
    switch (pl.radix[s]) {
      case 2: fft_stage<2, W, T, LW, INV>(buf, tw, pl.L, ns); break;
      case 3: fft_stage<3, W, T, LW, INV>(buf, tw, pl.L, ns); break;
      case 4: fft_stage<4, W, T, LW, INV>(buf, tw, pl.L, ns); break;
      case 5: fft_stage<5, W, T, LW, INV>(buf, tw, pl.L, ns); break;
      case 7: fft_stage<7, W, T, LW, INV>(buf, tw, pl.L, ns); break;
      case 8: fft_stage<8, W, T, LW, INV>(buf, tw, pl.L, ns); break;
      case 11: fft_stage<11, W, T, LW, INV>(buf, tw, pl.L, ns); break;
      default: break;
    }
  }
}

// ---------------------------------------------------------------- transform with fused I/O
// Fixed-length transform of W pencils whose first stage takes its inputs from a producer
// and whose last stage hands its outputs to a consumer, so that neither passes through LDS:
//   ld(i0, i1, p)       -> V        input element i0 + i1 of pencil p     (IN_LDS = false)
//   st(k0, k1, p, v, slot)         output element k0 + k1 of pencil p; slot is a compile-time
//                                  index (butterfly * R + t) unique per thread (OUT_LDS = false)
// The element index comes in two parts: i0 / k0 is the same for all R elements of a
// butterfly and i1 / k1 is a compile-time multiple of the stage stride, so a producer or
// consumer can form the per-butterfly part of an address once and add a uniform constant.
// With IN_LDS the first stage reads buf in natural order instead; with OUT_LDS the last
// stage writes buf in natural order instead.  buf must not be in use by other threads on
// entry (caller synchronises).  On return the group is NOT synchronised after the last
// stage; callers reusing buf (or reading it with OUT_LDS) must __syncthreads() first.
// The thread index behind an empty asm: index arithmetic derived from it cannot be hoisted
// out of callers' loops (which would keep dozens of addresses live across them).
__device__ __forceinline__ unsigned opaque_tid() {
  unsigned t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// A per-butterfly LDS index behind an empty asm: the R accesses of the butterfly then
// address buf[x + constant] with the constant in the instruction's offset field, instead of
// the compiler folding each constant into the index arithmetic (several ALU ops per access).
__device__ __forceinline__ unsigned opaque_idx(unsigned x) {
  asm volatile("" : "+v"(x));
  return x;
}

// The same without volatile: still opaque to constant folding, but the compiler may merge
// identical ones and schedule memory accesses across it (a volatile asm is a scheduling
// boundary, which serialises the LDS reads of consecutive butterflies).  For indices that
// derive from opaque_tid() or from loop variables, so nothing is hoisted out of loops.
__device__ __forceinline__ unsigned opaque_base(unsigned x) {
  asm("" : "+v"(x));
  return x;
}

template <int L, int R, int NS, int W, int WS, int WSO, int T, bool INV, bool FROM_LD, bool TO_ST, int NZ, typename LD,
          typename ST, typename V>
__device__ __forceinline__ void fft_stage_io(V* __restrict__ buf, const V* __restrict__ tw, LD& ld, ST& st) {
  const unsigned tx = opaque_tid();
  constexpr int LR = L / R;
  constexpr int NBF = LR * W;
  constexpr int NB = (NBF + T - 1) / T;
  auto finish = [&](V* v, unsigned p, unsigned j, int u) {
    const unsigned q = div_small<NS, LR>(j), k = j - mul24c<NS>(q);
    if constexpr (NS > 1) {
      // this butterfly's R - 1 factors are adjacent in the staged table
      const unsigned kb = opaque_base(mul24c<R - 1>(k));
#pragma unroll
      for (int t = 1; t < R; ++t) {
        V w = tw[kb + staged_tw_first<L, NS>() + t - 1];
        if (INV) w.y = -w.y;
        v[t] = cmul(v[t], w);
      }
    }
    dft<R, INV, NZ>(v);
    const unsigned base = mul24c<NS * R>(q) + k;
    if constexpr (TO_ST) {
#pragma unroll
      for (int t = 0; t < R; ++t) st(base, t * NS, p, v[t], u * R + t);
    } else {
      const unsigned wb = opaque_base(mul24c<WSO>(base) + p);
#pragma unroll
      for (int t = 0; t < R; ++t) buf[wb + t * NS * WSO] = v[t];
    }
  };
  if constexpr (FROM_LD || TO_ST) {
    // not in place (inputs come from the producer, or outputs go to the consumer): one
    // butterfly at a time keeps only R values live
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const unsigned bf = tx + u * T;
      if (NBF % T == 0 || bf < NBF) {
        const unsigned p = bf % W, j = bf / W;
        V v[R];
        if constexpr (FROM_LD) {
#pragma unroll
          for (int t = 0; t < R; ++t) v[t] = t < NZ ? ld(j, t * LR, p) : czero<V>();
        } else {
          const unsigned rb = opaque_base(mul24c<WS>(j) + p);
#pragma unroll
          for (int t = 0; t < R; ++t) v[t] = buf[rb + t * LR * WS];
        }
        finish(v, p, j, u);
      }
    }
  } else {
    // in place: every butterfly of the group is read before any is written
    V v[NB][R];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const unsigned bf = tx + u * T;
      if (NBF % T == 0 || bf < NBF) {
        const unsigned p = bf % W, j = bf / W;
        const unsigned rb = opaque_base(mul24c<WS>(j) + p);
#pragma unroll
        for (int t = 0; t < R; ++t) v[u][t] = buf[rb + t * LR * WS];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const unsigned bf = tx + u * T;
      if (NBF % T == 0 || bf < NBF) finish(v[u], bf % W, bf / W, u);
    }
  }
  if constexpr (!TO_ST) __syncthreads();
}

template <int L, int S, int W, int WS, int WSO, int T, bool INV, bool IN_LDS, bool OUT_LDS, bool HALF, typename LD,
          typename ST, typename V>
__device__ __forceinline__ void fft_io_stages(V* __restrict__ buf, const V* __restrict__ tw, LD& ld, ST& st) {
  constexpr CPlan P = make_cplan(L);
  if constexpr (S < P.nst) {
    constexpr bool first = (S == 0), last = (S + 1 == P.nst);
    // HALF: inputs i >= L/2 are zero, so the first stage's inputs t >= ceil(R/2) vanish
    constexpr int NZ = (first && HALF) ? (P.r[S] + 1) / 2 : P.r[S];
    // the last stage writes its LDS output with row stride WSO, every other write uses WS
    fft_stage_io<L, P.r[S], P.ns[S], W, WS, (last ? WSO : WS), T, INV, first && !IN_LDS, last && !OUT_LDS, NZ>(
        buf, tw, ld, st);
    fft_io_stages<L, S + 1, W, WS, WSO, T, INV, IN_LDS, OUT_LDS, HALF>(buf, tw, ld, st);
  }
}

// Call f(k, p, slot) for every output element a thread owns in the last stage of a
// fixed-length plan (same ownership and slot numbering as the consumer of fft_io).
template <int L, int W, int T, typename F>
__device__ __forceinline__ void for_each_last_slot(F&& f) {
  constexpr CPlan P = make_cplan(L);
  constexpr int R = P.r[P.nst - 1], NS = P.ns[P.nst - 1];
  constexpr int NBF = (L / R) * W, NB = (NBF + T - 1) / T;
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const unsigned bf = threadIdx.x + u * T;
    if (NBF % T == 0 || bf < NBF) {
      const unsigned p = bf % W, j = bf / W;
      const unsigned q = div_small<NS, L / R>(j), k = j - mul24c<NS>(q);
      const unsigned base = mul24c<NS * R>(q) + k;
#pragma unroll
      for (int t = 0; t < R; ++t) f(base + t * NS, p, u * R + t);
    }
  }
}

// Number of consumer slots per thread in the last stage of a fixed-length plan.
template <int L, int W, int T>
constexpr int last_slots() {
  constexpr CPlan P = make_cplan(L);
  constexpr int R = P.r[P.nst - 1];
  return ((L / R) * W + T - 1) / T * R;
}

// Consumer slots per thread for fft_io: the last stage's outputs (LC > 0) or the strided
// loop over the whole tile of the run-time path (LC == 0).
template <int LC, int W, int T>
constexpr int consumer_slots() {
  if constexpr (LC > 0) return last_slots<LC, W, T>();
  else return (kMaxLen * W + T - 1) / T;
}

// LC > 0: compile-time plan with fused I/O.  LC == 0: run-time plan: the producer fills buf,
// the LDS transform runs, and the consumer reads buf (slot = position in the thread's loop).
// WSO: row stride of the final LDS result (OUT_LDS), e.g. padded for a transposing reader.
// HALF (compile-time plans, producer input): the producer's inputs i >= L/2 are zero and
// are neither requested nor added.
template <int LC, int W, int T, bool INV, bool IN_LDS, bool OUT_LDS, int WSO = W, bool HALF = false, typename LD,
          typename ST, typename V>
__device__ __forceinline__ void fft_io(V* __restrict__ buf, const V* __restrict__ tw, const FftPlan& pl,
                                       LD&& ld, ST&& st) {
  static_assert(LC > 0 || WSO == W, "a padded result needs a compile-time plan");
  if constexpr (LC > 0) {
    fft_io_stages<LC, 0, W, W, WSO, T, INV, IN_LDS, OUT_LDS, HALF && !IN_LDS>(buf, tw, ld, st);
  } else {
    const int L = pl.L;
    if constexpr (!IN_LDS) {
      for (int e = threadIdx.x; e < L * W; e += T) buf[e] = ld(e / W, 0, e % W);
    }
    __syncthreads();
    fft_lds<W, T, INV>(buf, tw, pl);
    if constexpr (!OUT_LDS) {
      int slot = 0;
      for (int e = threadIdx.x; e < L * W; e += T, ++slot) st(e / W, 0, e % W, buf[e], slot);
    }
  }
}

// Lengths with a compile-time instance; every other supported length uses the run-time plan.
constexpr int kFastLengths[] = {16, 32, 48, 56, 64, 88, 96, 110, 128, 176, 192, 220, 256, 352, 440, 512};

// This length's twiddles into LDS (caller synchronises before use): the staged table of
// the compile-time plan (LC > 0), else the plain table w^i, i = 0 .. L - 1.  table + tw_off
// holds the plain table of the plan's length.
template <int LC, typename V>
__device__ __forceinline__ void load_twiddles(V* __restrict__ dst, const V* __restrict__ table, const FftPlan& pl) {
  const V* src = table + pl.tw_off;
  const int T = blockDim.x;
  if constexpr (LC > 0) {
    constexpr int N = staged_tw_size<LC>();
    for (int e = threadIdx.x; e < N; e += T) dst[e] = src[staged_tw_source<LC, 1>((unsigned)e)];
  } else {
    // two loads in flight per thread before either is stored (L <= 2 * blockDim.x in one pass)
    const int L = pl.L;
    for (int i = threadIdx.x; i < L; i += 2 * T) {
      const int j = i + T < L ? i + T : i;
      const V a = src[i], b = src[j];
      dst[i] = a;
      dst[j] = b;
    }
  }
}

}  // namespace csngf
