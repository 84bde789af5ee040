// Host runtime and C ABI of the CSNGF hot path (see include/csngf.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <random>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "csngf.h"
#include "csngf_debug.h"
#include "csngf_kernels.hpp"

using namespace csngf;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  const int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? CSNGF_E_OUT_OF_MEMORY
                                                                               : CSNGF_E_DEVICE;
  return fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr)                              \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

#define LAUNCHCHK(what)                                   \
  do {                                                    \
    hipError_t e_ = hipGetLastError();                    \
    if (e_ != hipSuccess) return hip_fail(e_, what);      \
  } while (0)

// ---------------------------------------------------------------- FFT plans
bool factor_plan(int L, FftPlan& pl) {
  if (L < 2 || L > kMaxLen) return false;
  std::memset(&pl, 0, sizeof(pl));
  int n = L, st = 0;
  const int odd[] = {11, 7, 5, 3};
  for (int r : odd)
    while (n % r == 0) {
      if (st >= kMaxStages) return false;
      pl.radix[st++] = r;
      n /= r;
    }
  while (n % 8 == 0) { pl.radix[st++] = 8; n /= 8; }
  while (n % 4 == 0) { pl.radix[st++] = 4; n /= 4; }
  while (n % 2 == 0) { pl.radix[st++] = 2; n /= 2; }
  if (n != 1) return false;
  pl.L = L;
  pl.nst = st;
  int ns = 1;
  for (int s = 0; s < st; ++s) {
    pl.ns[s] = ns;
    ns *= pl.radix[s];
  }
  return true;
}

bool supported(int L) {
  FftPlan pl;
  return L >= 8 && L <= kMaxLen && (L % 2) == 0 && factor_plan(L, pl);
}

int smallest_supported_at_least(int need) {
  for (int L = std::max(8, need); L <= kMaxLen; ++L)
    if (supported(L)) return L;
  return -1;
}

bool fast_length(int L) {
  for (int f : kFastLengths)
    if (f == L) return true;
  return false;
}

// Automatic FFT size: the smallest supported length >= need, unless it has no compile-time
// plan and one with a plan is at most 1.5x as long (the run-time-plan kernels are several
// times slower than the fixed-length ones, more than the extra padding costs).
int auto_pad(int need) {
  const int s0 = smallest_supported_at_least(need);
  if (s0 < 0 || fast_length(s0)) return s0;
  for (int L = s0 + 1; L <= kMaxLen && 2 * L <= 3 * s0; ++L)
    if (fast_length(L)) return L;
  return s0;
}

void twiddles(int L, std::vector<float2>& out) {
  for (int j = 0; j < L; ++j) {
    const double a = -2.0 * M_PI * (double)j / (double)L;
    out.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
  }
}

void twiddles(int L, std::vector<double2>& out) {
  for (int j = 0; j < L; ++j) {
    const double a = -2.0 * M_PI * (double)j / (double)L;
    out.push_back(make_double2(std::cos(a), std::sin(a)));
  }
}

size_t a16(size_t b) { return (b + 15) & ~size_t(15); }

// twiddles, transform rows, ring of 3 halo planes, NGF of one slice (+ Px floats of padding
// for the producer's reads past the last row)
size_t lds_fields(int Px, int nx, size_t el = sizeof(float2)) {
  return a16(el * Px) + a16(el * Px * (kRowsX + 1)) + a16(sizeof(float) * 3 * (kRowsX + 2) * nx) +
         a16(sizeof(float) * (3 * kRowsX * ng_stride(nx) + Px));
}

// slices per field-stage workgroup (z march); each new slice costs one resampled halo plane
#ifndef CSNGF_SLICES
#define CSNGF_SLICES 8
#endif
constexpr int kSlicesX = CSNGF_SLICES;
// final-pass workgroups walking the work list (8192 measured best of 1024 .. 16384 at 176^3/110^3)
constexpr int kFinalGroups = 8192;
size_t lds_pencil(int L, int W = kTileW, size_t el = sizeof(float2)) { return a16(el * L) + a16(el * L * W); }
size_t lds_final(int Px, int nxB, size_t el = sizeof(float2)) {
  return a16(el * Px) + a16(el * Px * (kRowsC + 1)) + a16(sizeof(int) * 2 * kRowsC * (nxB + 1));
}

// Call fn with std::integral_constant<int, L> for lengths that have a compile-time instance
// (kFastLengths) and std::integral_constant<int, 0> (run-time plan) otherwise.
template <typename Fn>
void with_len(int L, Fn&& fn) {
  switch (L) {
#define CSNGF_CASE(N)                          \
  case N:                                      \
    fn(std::integral_constant<int, N>{});      \
    return;
    CSNGF_CASE(16) CSNGF_CASE(32) CSNGF_CASE(48) CSNGF_CASE(56) CSNGF_CASE(64) CSNGF_CASE(88) CSNGF_CASE(96)
    CSNGF_CASE(110) CSNGF_CASE(128) CSNGF_CASE(176) CSNGF_CASE(192) CSNGF_CASE(220) CSNGF_CASE(256) CSNGF_CASE(352)
    CSNGF_CASE(440) CSNGF_CASE(512)
#undef CSNGF_CASE
    default:
      fn(std::integral_constant<int, 0>{});
      return;
  }
}

constexpr size_t kLdsDefault = 64 * 1024;
constexpr size_t kLdsMax = 160 * 1024;

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= kLdsDefault) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

int quantise(const double* R, int* k, double* Rq) {
  for (int i = 0; i < 9; ++i) {
    const double v = R[i];
    if (!std::isfinite(v) || std::fabs(v) > 2.0) return -1;
    const double q = std::nearbyint(v * 65536.0);  // round half to even (default mode)
    k[i] = (int)q;
    if (Rq) Rq[i] = q / 65536.0;
  }
  return 0;
}

bool all_finite(const float* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

enum KType { KT_FIELDS, KT_SAT, KT_YFWD, KT_ZPASS, KT_YINV, KT_FINAL, KT_MISC, KT_MASK, KT_COUNT };
const char* kTypeName[KT_COUNT] = {"fields_x", "overlap_sat", "y_forward", "z_mac_inverse",
                                   "y_inverse", "x_c2r_argmax", "misc", "overlap_fp64"};

struct PendingEv {
  int type;
  hipEvent_t a, b;
};

}  // namespace

struct csngf_ctx {
  int dev = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  int nA[3] = {0, 0, 0}, nB[3] = {0, 0, 0};  // x, y, z
  int P[3] = {0, 0, 0};
  int Wd[3] = {0, 0, 0};
  int H = 0, Hp = 0, tiles = 0;
  float eps = 1e-5f;
  double gamma = 0.5;
  uint32_t flags = 0;
  int nf = 6;  // separable fields: 6 (squared measure) or 3 (unsquared)
  int batch = 1;
  int slices = kSlicesX;            // z slices per field-stage workgroup
  int final_groups = kFinalGroups;  // final-pass workgroups without a map
  FftPlan plx{}, ply{}, plz{};
  float2* d_tw = nullptr;
  float2* d_spec = nullptr;
  long long spec_bytes = 0;
  long long count_a = 0;
  float2* d_buf1 = nullptr;
  float2* d_buf2 = nullptr;
  long long buf1_slot = 0, buf2_slot = 0;
  uint8_t* d_mask = nullptr;
  long long mask_slot = 0;
  int* d_sat = nullptr;
  long long sat_slot = 0;
  // per-slice 2-D prefix sums of the mask (SAT step 1), uint16 or uint32 per voxel
  uint32_t* d_plane = nullptr;
  long long plane_slot = 0;   // in uint32 units
  // the overlap table is built on a side stream, beside the y forward pass (both need only
  // the field stage's output), followed there by the packed-column z tiles, beside the main
  // z pass; fork after the field stage, join before the z pass and before the y inverse
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_yfwd = nullptr, ev_zpack = nullptr;
  uint8_t* d_flags = nullptr;
  long long flag_slot = 0;
  // the final pass's work list (active row groups) and its length at d_work[0]
  unsigned* d_work = nullptr;
  long long work_slot = 0;
  unsigned long long* d_keys = nullptr;
  RotResultDev* d_res = nullptr;
  int res_cap = 0;
  int* d_rot = nullptr;
  int rot_cap = 0;
  float* d_B = nullptr;
  float* d_Bb = nullptr;        // B in bricks of 4^3 cells (the moving side's gathers)
  long long brick_bytes = 0;
  uint8_t* d_mB = nullptr;
  int* d_flag = nullptr;
  RotResultDev* h_res = nullptr;
  int h_res_cap = 0;
  int* h_rot = nullptr;
  int h_rot_cap = 0;
  long long workspace_bytes = 0;
  // asynchronous evaluation in flight
  bool pending = false;
  int pend_n = 0;
  std::vector<int> pend_kq;
  hipEvent_t done_ev = nullptr;
  // graph replay of a full batch (CSNGF_GRAPHS)
  hipGraphExec_t gexec = nullptr;
  const float* g_B = nullptr;
  const uint8_t* g_mB = nullptr;
  int* d_rot_stage = nullptr;
  RotResultDev* d_res_stage = nullptr;
  bool prof = false;
  std::vector<PendingEv> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  long long stat_launches[KT_COUNT] = {0};
  double stat_ms[KT_COUNT] = {0};
  // kept displacement rows while profiling: [0] z-rows, [1] (z, y) rows; rotations counted
  unsigned long long* d_rowstat = nullptr;
  long long stat_rotations = 0;
  // a user mask on A: its eroded mask's bounding box (without one: [1, n_A - 2]), and the
  // FP64 chain that counts overlaps exactly
  bool masked = false;
  // CSNGF_FP64: the product fields are correlated in FP64 (buffers and spectra hold double2)
  bool fp64 = false;
  int lo[3] = {1, 1, 1}, hi[3] = {0, 0, 0};
  double2* d_twd = nullptr;     // FP64 twiddles, same offsets as d_tw
  double2* d_mspec = nullptr;   // conj of A's mask spectrum / (Px Py Pz), [Pz][Py][Hp]
  double2* d_mbuf1 = nullptr;   // per slot: X1m, then Y3m
  double2* d_mbuf2 = nullptr;   // per slot: X2m, then Y4m
  long long mbuf1_slot = 0, mbuf2_slot = 0;
  int* d_ncount = nullptr;      // per slot: exact N(chi), [Wz][Wy][Wx]
  long long ncount_slot = 0;
  uint8_t* d_ones = nullptr;    // every row flag set (full maps)
};

namespace {

hipError_t ev_get(csngf_ctx* c, hipEvent_t* e) {
  if (!c->ev_pool.empty()) {
    *e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Record a start event (profiling) before a launch; returns the event or nullptr.
hipEvent_t prof_begin(csngf_ctx* c, hipStream_t st = nullptr) {
  if (!c->prof) return nullptr;
  hipEvent_t e = nullptr;
  if (ev_get(c, &e) != hipSuccess) return nullptr;
  hipEventRecord(e, st ? st : c->stream);
  return e;
}

void prof_end(csngf_ctx* c, int type, hipEvent_t start, hipStream_t st = nullptr) {
  if (!start) return;
  hipEvent_t e = nullptr;
  if (ev_get(c, &e) != hipSuccess) return;
  hipEventRecord(e, st ? st : c->stream);
  c->prof_pending.push_back({type, start, e});
}

void prof_fold(csngf_ctx* c) {
  for (auto& p : c->prof_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->stat_ms[p.type] += ms;
      c->stat_launches[p.type] += 1;
    }
    c->ev_pool.push_back(p.a);
    c->ev_pool.push_back(p.b);
  }
  c->prof_pending.clear();
}

template <typename T>
void dfree(T*& p) {
  if (p) hipFree(p);
  p = nullptr;
}

template <typename T>
int dalloc(T** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(CSNGF_E_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                           hipGetErrorString(e));
  }
  return CSNGF_OK;
}

void release(csngf_ctx* c) {
  if (!c) return;
  hipSetDevice(c->dev);
  if (c->stream) hipStreamSynchronize(c->stream);
  if (c->side) hipStreamSynchronize(c->side);
  dfree(c->d_tw);
  dfree(c->d_spec);
  dfree(c->d_buf1);
  dfree(c->d_buf2);
  dfree(c->d_mask);
  dfree(c->d_sat);
  dfree(c->d_plane);
  dfree(c->d_work);
  dfree(c->d_flags);
  dfree(c->d_keys);
  dfree(c->d_res);
  dfree(c->d_rot);
  dfree(c->d_B);
  dfree(c->d_Bb);
  dfree(c->d_mB);
  dfree(c->d_flag);
  dfree(c->d_rot_stage);
  dfree(c->d_res_stage);
  dfree(c->d_rowstat);
  dfree(c->d_twd);
  dfree(c->d_mspec);
  dfree(c->d_mbuf1);
  dfree(c->d_mbuf2);
  dfree(c->d_ncount);
  dfree(c->d_ones);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->done_ev) (void)hipEventDestroy(c->done_ev);
  if (c->h_res) hipHostFree(c->h_res);
  if (c->h_rot) hipHostFree(c->h_rot);
  for (auto& p : c->prof_pending) {
    hipEventDestroy(p.a);
    hipEventDestroy(p.b);
  }
  for (auto e : c->ev_pool) hipEventDestroy(e);
  if (c->ev_fork) hipEventDestroy(c->ev_fork);
  if (c->ev_join) hipEventDestroy(c->ev_join);
  if (c->ev_yfwd) hipEventDestroy(c->ev_yfwd);
  if (c->ev_zpack) hipEventDestroy(c->ev_zpack);
  if (c->side) hipStreamDestroy(c->side);
  if (c->own_stream) hipStreamDestroy(c->own_stream);
  delete c;
}

int check_device() {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return fail(CSNGF_E_NO_DEVICE, "no HIP device visible");
  }
  return CSNGF_OK;
}

int check_dims(const csngf_dims& d, const char* what) {
  if (d.nx < 3 || d.ny < 3 || d.nz < 3)
    return fail(CSNGF_E_INVALID_ARG, std::string(what) + ": every extent must be >= 3");
  if (d.nx > kMaxLen || d.ny > kMaxLen || d.nz > kMaxLen)
    return fail(CSNGF_E_UNSUPPORTED, std::string(what) + ": extent above 512");
  return CSNGF_OK;
}

// Launch helpers -------------------------------------------------------------------------

template <typename V>
const V* twiddle_table(const csngf_ctx* c);
template <>
const float2* twiddle_table<float2>(const csngf_ctx* c) { return c->d_tw; }
template <>
const double2* twiddle_table<double2>(const csngf_ctx* c) { return c->d_twd; }

// The FP32 pencil passes of the product fields, or (double2) those of the exact overlap chain.
template <typename V>
int launch_pencil(csngf_ctx* c, bool inv, const V* in, V* out, int n_in, int n_out, int out_off,
                  const FftPlan& pl, long long in_g, long long out_g, int groups, long long in_s,
                  long long out_s, int slots, const uint8_t* flags = nullptr, long long flag_s = 0) {
  // tiles cover the H = Px/2 stored bins (bin 0 = DC + i Nyquist); the padding columns up to
  // Hp are never touched
  const int W = inv ? kTileP<true> : kTileP<false>;
  const dim3 grid((c->H + W - 1) / W, groups, slots);
  const size_t lds = lds_pencil(pl.L, W, sizeof(V)) + (inv ? a16(pl.L) : 0);   // + the inverse's row flags
  if (lds > kLdsMax) return fail(CSNGF_E_UNSUPPORTED, "FFT length too large for the pencil pass");
  hipError_t ae = hipSuccess;
  hipEvent_t ev = prof_begin(c);
  const bool half = 2 * n_in <= pl.L;  // inputs i >= L/2 are zero: first stage pruned
  with_len(pl.L, [&](auto lc) {
    constexpr int LC = decltype(lc)::value;
    auto go = [&](auto kern, int threads) {
      ae = allow_lds(kern, lds);
      if (ae == hipSuccess)
        hipLaunchKernelGGL(kern, grid, dim3(threads), lds, c->stream, in, out, n_in, n_out, out_off, pl,
                           twiddle_table<V>(c), c->H, c->Hp, in_g, out_g, in_s, out_s, flags, flag_s, groups);
    };
    if (inv) go(k_pencil<true, LC, false, V>, kThreadsP<true>);
    else if (half) go(k_pencil<false, LC, true, V>, kThreadsP<false>);
    else go(k_pencil<false, LC, false, V>, kThreadsP<false>);
  });
  prof_end(c, std::is_same<V, double2>::value ? KT_MASK : inv ? KT_YINV : KT_YFWD, ev);
  if (ae != hipSuccess) return hip_fail(ae, "hipFuncSetAttribute(k_pencil)");
  LAUNCHCHK(inv ? "k_pencil<inverse>" : "k_pencil<forward>");
  return CSNGF_OK;
}

// z pass over the slots' X2 tiles: per field the z forward, the MAC against A's conjugate
// spectra, then the z inverse of the sum, storing the kept z-rows.  The two tiles that hold the
// packed DC/Nyquist column go to pack_stream (the side stream for the product fields), the
// rest to the context's stream.
template <typename V>
int launch_zpass(csngf_ctx* c, const V* X2, const V* spec, V* Y3, int nf, long long x2_slot, long long y3_slot,
                 const uint8_t* flags, long long flag_slot, int slots, hipStream_t pack_stream) {
  const int nreal = c->P[1] * c->tiles * slots;
  const int nb8 = (nreal + 7) / 8 * 8;
  const size_t lds = lds_pencil(c->plz.L, kTileW, sizeof(V)) + a16(c->plz.L);   // + the kept-row flags
  if (lds > kLdsMax) return fail(CSNGF_E_UNSUPPORTED, "FFT length too large for the z pass");
  const int out_off = c->P[2] - (c->nA[2] - 1);
  hipError_t ae = hipSuccess;
  hipEvent_t ev = prof_begin(c);
  // inputs z >= Pz/2 are zero when nz - 2 <= Pz/2: the forward transforms' first stage is pruned
  const bool half = 2 * (c->nB[2] - 2) <= c->plz.L;
  with_len(c->plz.L, [&](auto lc) {
    constexpr int LC = decltype(lc)::value;
    auto go = [&](auto kern, int nblocks, hipStream_t st) {
      if (ae == hipSuccess) ae = allow_lds(kern, lds);
      if (ae == hipSuccess)
        hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kThreadsZ), lds, st, X2, spec, Y3, c->nB[2] - 2, c->P[1], c->H,
                           c->Hp, c->Wd[2], out_off, c->plz, twiddle_table<V>(c), x2_slot, y3_slot, c->tiles, slots,
                           nreal, flags, flag_slot, nf);
    };
    if (half) {
      go(k_zpass<LC, true, true, V>, 2 * slots, pack_stream);
      go(k_zpass<LC, true, false, V>, nb8, c->stream);
    } else {
      go(k_zpass<LC, false, true, V>, 2 * slots, pack_stream);
      go(k_zpass<LC, false, false, V>, nb8, c->stream);
    }
  });
  prof_end(c, std::is_same<V, double2>::value ? KT_MASK : KT_ZPASS, ev);
  if (ae != hipSuccess) return hip_fail(ae, "hipFuncSetAttribute(k_zpass)");
  LAUNCHCHK("k_zpass");
  return CSNGF_OK;
}

// Field stage of `slots` volumes: FP32 NGF and products, x transform in V (float2, or double2
// for CSNGF_FP64); dbg (FP32 only) also copies the products out.
template <typename V>
int launch_fields(csngf_ctx* c, bool moving, const float* vol, const uint8_t* um, const int* n3, const int* rotq,
                  V* out, long long out_slot, uint8_t* mask_out, long long mask_slot, float* dbg, int slots) {
  const int tz = c->slices;
  const int nreal = (n3[1] + kRowsX - 1) / kRowsX * ((n3[2] + tz - 1) / tz) * slots;
  const dim3 grid((nreal + 7) / 8 * 8);
  const size_t lds = lds_fields(c->plx.L, n3[0], sizeof(V));
  if (lds > kLdsMax) return fail(CSNGF_E_UNSUPPORTED, "x extent too large for the field stage");
  hipError_t ae = hipSuccess;
  hipEvent_t ev = prof_begin(c);
  // inputs x >= Px/2 are zero when nx <= Px/2: the transform's first stage is pruned
  const bool half = 2 * n3[0] <= c->plx.L;
  auto go = [&](auto kern) {
    ae = allow_lds(kern, lds);
    if (ae == hipSuccess)
      hipLaunchKernelGGL(kern, grid, dim3(kThreadsF), lds, c->stream, vol, um, n3[0], n3[1], n3[2], tz, slots, c->nf,
                         rotq, c->eps, c->plx, twiddle_table<V>(c), out, c->H, c->Hp, out_slot, mask_out, mask_slot, dbg);
  };
  bool done = false;
  if constexpr (std::is_same<V, float2>::value) {
    if (dbg) {   // the debug copy of the products: the run-time-plan instance
      if (moving) {
        if (half) go(k_fields_x<true, 0, true, true>);
        else go(k_fields_x<true, 0, false, true>);
      } else {
        if (half) go(k_fields_x<false, 0, true, true>);
        else go(k_fields_x<false, 0, false, true>);
      }
      done = true;
    }
  }
  if (!done) {
    with_len(c->plx.L, [&](auto lc) {
      constexpr int LC = decltype(lc)::value;
      if (moving) {
        if (half) go(k_fields_x<true, LC, true, false, V>);
        else go(k_fields_x<true, LC, false, false, V>);
      } else {
        if (half) go(k_fields_x<false, LC, true, false, V>);
        else go(k_fields_x<false, LC, false, false, V>);
      }
    });
  }
  prof_end(c, KT_FIELDS, ev);
  if (ae != hipSuccess) return hip_fail(ae, "hipFuncSetAttribute(k_fields_x)");
  LAUNCHCHK("k_fields_x");
  return CSNGF_OK;
}

OverlapGeom geometry(const csngf_ctx* c) {
  OverlapGeom g;
  for (int i = 0; i < 3; ++i) {
    g.nA[i] = c->nA[i];
    g.nB[i] = c->nB[i];
    g.lo[i] = c->lo[i];
    g.hi[i] = c->hi[i];
  }
  return g;
}

// The exact overlap chain of a fixed side with a general mask (FP64): the eroded moving masks
// of the slots -> x R2C -> y forward -> z forward x conj(A's mask spectrum) -> z inverse ->
// y inverse -> x C2R, rounded into d_ncount.  flags: the kept rows (all ones for a full map).
int run_overlap_chain(csngf_ctx* c, int slots, const uint8_t* flags, long long flag_slot) {
  const int nx = c->nB[0], ny = c->nB[1], nz = c->nB[2];
  {
    const size_t lds = a16(sizeof(double2) * c->plx.L) + a16(sizeof(double2) * c->plx.L * kMaskPairs);
    if (lds > kLdsMax) return fail(CSNGF_E_UNSUPPORTED, "x extent too large for the overlap chain");
    const dim3 grid(((ny - 2 + 1) / 2 + kMaskPairs - 1) / kMaskPairs, nz - 2, slots);
    const bool half = 2 * nx <= c->plx.L;
    hipError_t ae = hipSuccess;
    hipEvent_t ev = prof_begin(c);
    with_len(c->plx.L, [&](auto lc) {
      constexpr int LC = decltype(lc)::value;
      auto go = [&](auto kern) {
        ae = allow_lds(kern, lds);
        if (ae == hipSuccess)
          hipLaunchKernelGGL(kern, grid, dim3(kThreadsM), lds, c->stream, c->d_mask, nx, ny, nz, c->mask_slot, c->plx,
                             c->d_twd, c->d_mbuf1, c->H, c->Hp, c->mbuf1_slot);
      };
      if (half) go(k_mask_x<LC, true>);
      else go(k_mask_x<LC, false>);
    });
    prof_end(c, KT_MASK, ev);
    if (ae != hipSuccess) return hip_fail(ae, "hipFuncSetAttribute(k_mask_x)");
    LAUNCHCHK("k_mask_x");
  }
  int rc = launch_pencil(c, false, c->d_mbuf1, c->d_mbuf2, ny - 2, c->P[1], 0, c->ply, (long long)(ny - 2) * c->Hp,
                         (long long)c->P[1] * c->Hp, nz - 2, c->mbuf1_slot, c->mbuf2_slot, slots);
  if (rc) return rc;
  rc = launch_zpass(c, c->d_mbuf2, c->d_mspec, c->d_mbuf1, 1, c->mbuf2_slot, c->mbuf1_slot, flags, flag_slot, slots,
                    c->stream);
  if (rc) return rc;
  rc = launch_pencil(c, true, c->d_mbuf1, c->d_mbuf2, c->P[1], c->Wd[1], c->P[1] - (c->nA[1] - 1), c->ply,
                     (long long)c->P[1] * c->Hp, (long long)c->Wd[1] * c->Hp, c->Wd[2], c->mbuf1_slot, c->mbuf2_slot,
                     slots, flags, flag_slot);
  if (rc) return rc;
  {
    const size_t lds = a16(sizeof(double2) * c->plx.L) + a16(sizeof(double2) * c->plx.L * (kRowsC + 1));
    if (lds > kLdsMax) return fail(CSNGF_E_UNSUPPORTED, "x extent too large for the overlap chain");
    const dim3 grid((c->Wd[1] + 2 * kRowsC - 1) / (2 * kRowsC), c->Wd[2], slots);
    hipError_t ae = hipSuccess;
    hipEvent_t ev = prof_begin(c);
    with_len(c->plx.L, [&](auto lc) {
      constexpr int LC = decltype(lc)::value;
      ae = allow_lds(k_overlap_x<LC>, lds);
      if (ae == hipSuccess)
        hipLaunchKernelGGL((k_overlap_x<LC>), grid, dim3(kThreadsC), lds, c->stream, c->d_mbuf2, c->d_ncount, c->Wd[0],
                           c->Wd[1], c->Wd[2], c->H, c->Hp, c->nA[0] - 1, c->plx, c->d_twd, c->mbuf2_slot,
                           c->ncount_slot, flags, flag_slot);
    });
    prof_end(c, KT_MASK, ev);
    if (ae != hipSuccess) return hip_fail(ae, "hipFuncSetAttribute(k_overlap_x)");
    LAUNCHCHK("k_overlap_x");
  }
  return CSNGF_OK;
}

// A's side of the overlap chain: its eroded mask meff (device, dims nA) -> count and bounding
// box (host) -> FP64 x R2C, y forward, z forward -> d_mspec = conj(.) / (Px Py Pz).
int fixed_mask_spectrum(csngf_ctx* c, const uint8_t* meff, const int* nA) {
  const size_t nvA = (size_t)nA[0] * nA[1] * nA[2];
  {
    // the field stage wrote meff on the context's stream, which is non-blocking: a plain
    // hipMemcpy would not wait for it
    std::vector<uint8_t> h(nvA);
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(h.data(), meff, nvA, hipMemcpyDeviceToHost));
    long long cnt = 0;
    int lo[3] = {nA[0], nA[1], nA[2]}, hi[3] = {-1, -1, -1};
    for (int z = 0; z < nA[2]; ++z)
      for (int y = 0; y < nA[1]; ++y)
        for (int x = 0; x < nA[0]; ++x)
          if (h[((size_t)z * nA[1] + y) * nA[0] + x]) {
            ++cnt;
            const int v[3] = {x, y, z};
            for (int i = 0; i < 3; ++i) {
              lo[i] = std::min(lo[i], v[i]);
              hi[i] = std::max(hi[i], v[i]);
            }
          }
    c->count_a = cnt;
    for (int i = 0; i < 3; ++i) {
      c->lo[i] = cnt ? lo[i] : 1;   // an empty mask: lo > hi, every bound is 0
      c->hi[i] = cnt ? hi[i] : 0;
    }
  }
  const int* P = c->P;
  const long long Hp = c->Hp;
  double2 *x1m = nullptr, *x2m = nullptr;
  int rc = dalloc(&x1m, sizeof(double2) * (size_t)(nA[2] - 2) * (nA[1] - 2) * Hp);
  if (!rc) rc = dalloc(&x2m, sizeof(double2) * (size_t)(nA[2] - 2) * P[1] * Hp);
  if (!rc) {
    const size_t lds = a16(sizeof(double2) * c->plx.L) + a16(sizeof(double2) * c->plx.L * kMaskPairs);
    const dim3 grid(((nA[1] - 2 + 1) / 2 + kMaskPairs - 1) / kMaskPairs, nA[2] - 2, 1);
    const bool half = 2 * nA[0] <= c->plx.L;
    hipError_t ae = hipSuccess;
    with_len(c->plx.L, [&](auto lc) {
      constexpr int LC = decltype(lc)::value;
      auto go = [&](auto kern) {
        ae = allow_lds(kern, lds);
        if (ae == hipSuccess)
          hipLaunchKernelGGL(kern, grid, dim3(kThreadsM), lds, c->stream, meff, nA[0], nA[1], nA[2], 0LL, c->plx,
                             c->d_twd, x1m, c->H, c->Hp, 0LL);
      };
      if (lds > kLdsMax) ae = hipErrorInvalidValue;
      else if (half) go(k_mask_x<LC, true>);
      else go(k_mask_x<LC, false>);
    });
    if (ae != hipSuccess) rc = hip_fail(ae, "k_mask_x (fixed side)");
    else if (hipGetLastError() != hipSuccess) rc = fail(CSNGF_E_DEVICE, "k_mask_x (fixed side) launch");
  }
  if (!rc)
    rc = launch_pencil(c, false, x1m, x2m, nA[1] - 2, P[1], 0, c->ply, (long long)(nA[1] - 2) * Hp,
                       (long long)P[1] * Hp, nA[2] - 2, 0, 0, 1);
  if (!rc) rc = dalloc(&c->d_mspec, sizeof(double2) * (size_t)P[2] * P[1] * Hp);
  if (!rc) {
    const double scale = 1.0 / ((double)P[0] * (double)P[1] * (double)P[2]);
    const dim3 grid(c->tiles, P[1], 1);
    const size_t lds = lds_pencil(P[2], kTileW, sizeof(double2));
    hipError_t ae = hipSuccess;
    with_len(P[2], [&](auto lc) {
      constexpr int LC = decltype(lc)::value;
      ae = allow_lds(k_zstore<LC, double2>, lds);
      if (ae == hipSuccess)
        hipLaunchKernelGGL((k_zstore<LC, double2>), grid, dim3(kThreads), lds, c->stream, x2m, c->d_mspec, nA[2] - 2,
                           P[1], c->H, c->Hp, c->plz, c->d_twd, scale, 1);
    });
    if (ae != hipSuccess) rc = hip_fail(ae, "k_zstore (mask)");
    else if (hipGetLastError() != hipSuccess) rc = fail(CSNGF_E_DEVICE, "k_zstore (mask) launch");
  }
  const hipError_t se = hipStreamSynchronize(c->stream);
  if (!rc && se != hipSuccess) rc = hip_fail(se, "fixed-side mask spectrum");
  if (x1m) hipFree(x1m);
  if (x2m) hipFree(x2m);
  return rc;
}

// One launch sequence over `slots` rotations whose Q16 tables start at rotq (device).
template <typename V>
int run_batch_t(csngf_ctx* c, const float* dB, const uint8_t* dmB, const int* rotq, int slots, RotResultDev* res,
                float* cmap, long long* nmap) {
  int rc;
  hipEvent_t ev;
  V* buf1 = reinterpret_cast<V*>(c->d_buf1);
  V* buf2 = reinterpret_cast<V*>(c->d_buf2);
  const V* spec = reinterpret_cast<const V*>(c->d_spec);
  // Overlap table on the side stream (it also clears the per-slot argmax keys, before the join).
  // Without a user mask on B or A the moving masks are runs found from the rotations alone, so
  // the table is built beside the field stage; otherwise the field stage writes the masks and
  // the table is built from them beside the y forward pass.  The fork comes after the previous
  // sequence's last reader of the masks, table, flags and work list on this stream.
  const bool runs = dmB == nullptr && !c->masked;
  auto overlap_table = [&]() -> int {
    HIPCHK(hipEventRecord(c->ev_fork, c->stream));
    HIPCHK(hipStreamWaitEvent(c->side, c->ev_fork, 0));
    const int nx = c->nB[0], ny = c->nB[1], nz = c->nB[2];
    hipStream_t st = c->side;
    hipEvent_t e = prof_begin(c, st);
    int2* d_runs = reinterpret_cast<int2*>(c->d_mask);   // the mask slots hold the runs instead
    const long long runs_slot = c->mask_slot / (long long)sizeof(int2);
    if (runs)
      hipLaunchKernelGGL(k_mask_runs, dim3((ny * nz + kThreads - 1) / kThreads, slots), dim3(kThreads), 0, st, rotq,
                         nx, ny, nz, d_runs, runs_slot);
    const dim3 gz(((nx + 1) * (ny + 1) + kThreads - 1) / kThreads, slots);
    const dim3 gp((nx + 63) / 64, nz, slots);
    if ((long long)nx * ny < 65536) {   // 2-D prefix sums fit 16 bits
      uint16_t* pl16 = reinterpret_cast<uint16_t*>(c->d_plane);
      if (runs)
        hipLaunchKernelGGL(k_sat_planes_runs<uint16_t>, gp, dim3(64), 0, st, d_runs, pl16, nx, ny, runs_slot,
                           2 * c->plane_slot);
      else
        hipLaunchKernelGGL(k_sat_planes<uint16_t>, dim3(nz, slots), dim3(kSatThreads), 0, st, c->d_mask, pl16, nx,
                           ny, c->mask_slot, 2 * c->plane_slot);
      hipLaunchKernelGGL(k_sat_z<uint16_t>, gz, dim3(kThreads), 0, st, pl16, c->d_sat, nx, ny, nz, 2 * c->plane_slot,
                         c->sat_slot);
    } else {
      if (runs)
        hipLaunchKernelGGL(k_sat_planes_runs<uint32_t>, gp, dim3(64), 0, st, d_runs, c->d_plane, nx, ny, runs_slot,
                           c->plane_slot);
      else
        hipLaunchKernelGGL(k_sat_planes<uint32_t>, dim3(nz, slots), dim3(kSatThreads), 0, st, c->d_mask, c->d_plane,
                           nx, ny, c->mask_slot, c->plane_slot);
      hipLaunchKernelGGL(k_sat_z<uint32_t>, gz, dim3(kThreads), 0, st, c->d_plane, c->d_sat, nx, ny, nz,
                         c->plane_slot, c->sat_slot);
    }
    const OverlapGeom g = geometry(c);
    hipLaunchKernelGGL(k_bounds, dim3((c->Wd[2] * c->Wd[1] + kThreads - 1) / kThreads, slots), dim3(kThreads), 0,
                       st, c->d_sat, g, c->Wd[1], c->Wd[2], c->sat_slot, c->count_a, c->gamma, c->d_flags,
                       c->flag_slot, c->d_keys, c->d_work, c->prof ? c->d_rowstat : nullptr);
    if (c->prof) c->stat_rotations += slots;
    {
      const int items = slots * c->Wd[2] * ((c->Wd[1] + 2 * kRowsC - 1) / (2 * kRowsC));
      hipLaunchKernelGGL(k_worklist, dim3((items + kThreads - 1) / kThreads), dim3(kThreads), 0, st, c->d_flags,
                         c->flag_slot, c->Wd[1], c->Wd[2], 2 * kRowsC, slots, c->d_work + 64, c->d_work);
    }
    prof_end(c, KT_SAT, e, st);
    LAUNCHCHK("k_sat");
    HIPCHK(hipEventRecord(c->ev_join, st));
    return CSNGF_OK;
  };
  if (runs && (rc = overlap_table())) return rc;
  rc = launch_fields(c, true, dB, dmB, c->nB, rotq, buf1, c->buf1_slot, runs ? nullptr : c->d_mask, c->mask_slot,
                     nullptr, slots);
  if (rc) return rc;
  if (!runs && (rc = overlap_table())) return rc;
  // y forward: X1 [slot][f][z][y] -> X2 [slot][f][z][ky]
  // (X1 holds the interior rows and slices only: the fields vanish on the border planes)
  rc = launch_pencil(c, false, buf1, buf2, c->nB[1] - 2, c->P[1], 0, c->ply,
                     (long long)(c->nB[1] - 2) * c->Hp, (long long)c->P[1] * c->Hp, c->nf * (c->nB[2] - 2),
                     c->buf1_slot, c->buf2_slot, slots);
  if (rc) return rc;
  // the packed-column z tiles (2 workgroups per slot) go to the side stream, after the overlap
  // table there and the y forward here; the main z pass reads the kept-row flags, so it
  // waits for the table; the y inverse waits for both z launches
  HIPCHK(hipEventRecord(c->ev_yfwd, c->stream));
  HIPCHK(hipStreamWaitEvent(c->side, c->ev_yfwd, 0));
  HIPCHK(hipStreamWaitEvent(c->stream, c->ev_join, 0));
  // the packed DC/Nyquist tiles (tile 0 at ky = 0 and Py/2) on the side stream, all other
  // tiles here
  rc = launch_zpass(c, buf2, spec, buf1, c->nf, c->buf2_slot, c->buf1_slot, c->d_flags, c->flag_slot, slots, c->side);
  if (rc) return rc;
  HIPCHK(hipEventRecord(c->ev_zpack, c->side));
  HIPCHK(hipStreamWaitEvent(c->stream, c->ev_zpack, 0));
  // y inverse: Y3 [slot][zc][ky] -> Y4 [slot][zc][yc]
  rc = launch_pencil(c, true, buf1, buf2, c->P[1], c->Wd[1], c->P[1] - (c->nA[1] - 1), c->ply,
                     (long long)c->P[1] * c->Hp, (long long)c->Wd[1] * c->Hp, c->Wd[2], c->buf1_slot, c->buf2_slot,
                     slots, c->d_flags, c->flag_slot);
  if (rc) return rc;
  // a fixed side with a general mask: exact counts from the FP64 overlap chain (every row for
  // a full map, the kept rows otherwise)
  if (c->masked && (rc = run_overlap_chain(c, slots, cmap ? c->d_ones : c->d_flags, cmap ? 0 : c->flag_slot)))
    return rc;
  {
    const OverlapGeom g = geometry(c);
    const int* ncount = c->masked ? c->d_ncount : nullptr;
    const dim3 grid((c->Wd[1] + 2 * kRowsC - 1) / (2 * kRowsC), c->Wd[2], slots);
    // without a map: a fixed grid over the work list of row groups that hold a valid
    // displacement (most do not at gamma = 0.5)
    const int items = (int)(grid.x * grid.y * grid.z);
    const dim3 lgrid(std::min(items, c->final_groups));
    const size_t lds = lds_final(c->plx.L, c->nB[0], sizeof(V));
    hipError_t ae = hipSuccess;
    ev = prof_begin(c);
    with_len(c->plx.L, [&](auto lc) {
      constexpr int LC = decltype(lc)::value;
      auto go = [&](auto kern, dim3 gr, const unsigned* work, const unsigned* nwork) {
        ae = allow_lds(kern, lds);
        if (ae == hipSuccess)
          hipLaunchKernelGGL(kern, gr, dim3(kThreadsC), lds, c->stream, buf2, c->d_sat, c->d_keys, g, c->Wd[0],
                             c->Wd[1], c->Wd[2], c->H, c->Hp, c->plx, twiddle_table<V>(c), c->buf2_slot, c->sat_slot,
                             c->count_a, c->gamma, cmap, nmap, c->d_flags, c->flag_slot, work, nwork, ncount,
                             c->ncount_slot);
      };
      // with a map every row group gets a workgroup; without, a fixed grid walks the work list
      if (cmap && ncount) go(k_final_x<true, LC, true, V>, grid, nullptr, nullptr);
      else if (cmap) go(k_final_x<true, LC, false, V>, grid, nullptr, nullptr);
      else if (ncount) go(k_final_x<false, LC, true, V>, lgrid, c->d_work + 64, c->d_work);
      else go(k_final_x<false, LC, false, V>, lgrid, c->d_work + 64, c->d_work);
    });
    if (ae != hipSuccess) return hip_fail(ae, "hipFuncSetAttribute(k_final_x)");
    prof_end(c, KT_FINAL, ev);
    LAUNCHCHK("k_final_x");
    ev = prof_begin(c);
    hipLaunchKernelGGL(k_finalize, dim3((slots + 63) / 64), dim3(64), 0, c->stream, c->d_keys, c->d_sat, g, c->Wd[0],
                       c->Wd[1], c->sat_slot, slots, res, ncount, c->ncount_slot);
    prof_end(c, KT_MISC, ev);
    LAUNCHCHK("k_finalize");
  }
  return CSNGF_OK;
}

// A's side: fields (with its eroded mask written to meff when given), y forward, z forward
// stored as w_f conj(.) / (Px Py Pz) in d_spec, in the context's precision V.
template <typename V>
int fixed_spectra(csngf_ctx* c, const float* dA, const uint8_t* dmA, const int* nA, uint8_t* meff) {
  using S = scalar_t<V>;
  const int* P = c->P;
  const long long Hp = c->Hp;
  V *x1 = nullptr, *x2 = nullptr;
  const long long x1e = (long long)c->nf * nA[2] * nA[1] * Hp, x2e = (long long)c->nf * nA[2] * P[1] * Hp;
  int rc = dalloc(&x1, sizeof(V) * x1e);
  if (!rc) rc = dalloc(&x2, sizeof(V) * x2e);
  if (!rc) rc = launch_fields(c, false, dA, dmA, nA, nullptr, x1, 0, meff, 0, nullptr, 1);
  if (!rc)
    rc = launch_pencil(c, false, x1, x2, nA[1] - 2, P[1], 0, c->ply, (long long)(nA[1] - 2) * Hp, (long long)P[1] * Hp,
                       c->nf * (nA[2] - 2), 0, 0, 1);
  if (!rc) {
    const S scale = (S)(1.0 / ((double)P[0] * (double)P[1] * (double)P[2]));
    const dim3 grid(c->tiles, P[1], c->nf);
    const size_t lds = lds_pencil(P[2], kTileW, sizeof(V));
    hipError_t ae = hipSuccess;
    with_len(P[2], [&](auto lc) {
      constexpr int LC = decltype(lc)::value;
      ae = allow_lds(k_zstore<LC, V>, lds);
      if (ae == hipSuccess)
        hipLaunchKernelGGL((k_zstore<LC, V>), grid, dim3(kThreads), lds, c->stream, x2, reinterpret_cast<V*>(c->d_spec),
                           nA[2] - 2, P[1], c->H, c->Hp, c->plz, twiddle_table<V>(c), scale, c->nf);
    });
    const hipError_t e = ae != hipSuccess ? ae : hipGetLastError();
    if (e != hipSuccess) rc = hip_fail(e, "k_zstore");
  }
  const hipError_t se = hipStreamSynchronize(c->stream);
  if (!rc && se != hipSuccess) rc = hip_fail(se, "fixed-side precompute");
  if (x1) hipFree(x1);
  if (x2) hipFree(x2);
  return rc;
}

// One launch sequence in the context's precision.
int run_batch(csngf_ctx* c, const float* dB, const uint8_t* dmB, const int* rotq, int slots, RotResultDev* res,
              float* cmap, long long* nmap) {
  return c->fp64 ? run_batch_t<double2>(c, dB, dmB, rotq, slots, res, cmap, nmap)
                 : run_batch_t<float2>(c, dB, dmB, rotq, slots, res, cmap, nmap);
}

// A full batch through a captured graph: the launch sequence of run_batch is recorded once
// (reading rotations from, and writing results to, fixed staging slots) and replayed; it is
// re-recorded when the moving volume's device pointers change.
int run_graph_batch(csngf_ctx* c, const float* dB, const uint8_t* dmB, int base) {
  if (!c->gexec || c->g_B != dB || c->g_mB != dmB) {
    if (c->gexec) {
      (void)hipGraphExecDestroy(c->gexec);
      c->gexec = nullptr;
    }
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = run_batch(c, dB, dmB, c->d_rot_stage, c->batch, c->d_res_stage, nullptr, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->gexec = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
    c->g_B = dB;
    c->g_mB = dmB;
  }
  HIPCHK(hipMemcpyAsync(c->d_rot_stage, c->d_rot + 9 * (size_t)base, sizeof(int) * 9 * (size_t)c->batch,
                        hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(hipGraphLaunch(c->gexec, c->stream));
  HIPCHK(hipMemcpyAsync(c->d_res + base, c->d_res_stage, sizeof(RotResultDev) * (size_t)c->batch,
                        hipMemcpyDeviceToDevice, c->stream));
  return CSNGF_OK;
}


int ensure_rot_capacity(csngf_ctx* c, int n) {
  if (n <= c->rot_cap && n <= c->h_rot_cap && n <= c->res_cap && n <= c->h_res_cap) return CSNGF_OK;
  const int cap = std::max(n, 64);
  dfree(c->d_rot);
  dfree(c->d_res);
  if (c->h_rot) hipHostFree(c->h_rot);
  if (c->h_res) hipHostFree(c->h_res);
  c->h_rot = nullptr;
  c->h_res = nullptr;
  c->rot_cap = c->res_cap = c->h_rot_cap = c->h_res_cap = 0;
  int rc = dalloc(&c->d_rot, sizeof(int) * 9 * (size_t)cap);
  if (rc) return rc;
  rc = dalloc(&c->d_res, sizeof(RotResultDev) * (size_t)cap);
  if (rc) return rc;
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&c->h_rot), sizeof(int) * 9 * (size_t)cap));
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&c->h_res), sizeof(RotResultDev) * (size_t)cap));
  c->rot_cap = c->res_cap = c->h_rot_cap = c->h_res_cap = cap;
  return CSNGF_OK;
}

// B's copy in bricks (k_brick): values per volume, and the launch
long long brick_floats(const int* n3) {
  return (long long)kBrickVals * brick_count(n3[0]) * brick_count(n3[1]) * brick_count(n3[2]);
}

int launch_brick(hipStream_t s, const float* vol, const int* n3, float* out) {
  const long long total = brick_floats(n3);
  hipLaunchKernelGGL(k_brick, dim3((unsigned)((total + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, vol, n3[0],
                     n3[1], n3[2], out, total);
  LAUNCHCHK("k_brick");
  return CSNGF_OK;
}

// Stage the moving volume (and mask) on the device; device-pointer inputs are checked for
// non-finite values by a kernel whose flag is read after the call's final synchronisation.
int stage_moving(csngf_ctx* c, const float* B, const uint8_t* maskB, const float** dB, const uint8_t** dmB) {
  const size_t nv = (size_t)c->nB[0] * c->nB[1] * c->nB[2];
  if (c->flags & CSNGF_DEVICE_PTRS) {
    *dB = B;
    *dmB = maskB;
    HIPCHK(hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
    hipLaunchKernelGGL(k_check_finite, dim3(1024), dim3(256), 0, c->stream, B, (long long)nv, c->d_flag);
    LAUNCHCHK("k_check_finite");
    *dB = c->d_Bb;   // the field stage gathers from the brick copy
    return launch_brick(c->stream, B, c->nB, c->d_Bb);
  }
  if (!all_finite(B, nv)) return fail(CSNGF_E_INVALID_ARG, "moving volume B has a non-finite value");
  if (!c->d_B) {
    int rc = dalloc(&c->d_B, sizeof(float) * nv);
    if (rc) return rc;
  }
  HIPCHK(hipMemcpyAsync(c->d_B, B, sizeof(float) * nv, hipMemcpyHostToDevice, c->stream));
  int brc = launch_brick(c->stream, c->d_B, c->nB, c->d_Bb);
  if (brc) return brc;
  *dB = c->d_Bb;   // the field stage gathers from the brick copy
  *dmB = nullptr;
  if (maskB) {
    if (!c->d_mB) {
      int rc = dalloc(&c->d_mB, nv);
      if (rc) return rc;
    }
    HIPCHK(hipMemcpyAsync(c->d_mB, maskB, nv, hipMemcpyHostToDevice, c->stream));
    *dmB = c->d_mB;
  }
  return CSNGF_OK;
}

int read_flag(csngf_ctx* c, int* bad) {
  *bad = 0;
  if (!(c->flags & CSNGF_DEVICE_PTRS)) return CSNGF_OK;
  HIPCHK(hipMemcpy(bad, c->d_flag, sizeof(int), hipMemcpyDeviceToHost));
  return CSNGF_OK;
}

}  // namespace

// =================================================================================== ABI
extern "C" {

const char* csngf_last_error(void) { return g_err.c_str(); }

int csngf_default_params(csngf_params* out) {
  if (!out) return fail(CSNGF_E_INVALID_ARG, "params is NULL");
  std::memset(out, 0, sizeof(*out));
  out->struct_size = sizeof(csngf_params);
  out->eps = 1e-5f;
  out->gamma = 0.5;
  return CSNGF_OK;
}

int csngf_supported_length(int32_t L) { return supported(L) ? 1 : 0; }

int csngf_create(const float* A, csngf_dims dA, const uint8_t* maskA, csngf_dims dB, const csngf_params* p,
                 csngf_ctx** out) {
  if (!out) return fail(CSNGF_E_INVALID_ARG, "out is NULL");
  if (!A) return fail(CSNGF_E_INVALID_ARG, "fixed volume A is NULL");
  csngf_params prm;
  csngf_default_params(&prm);
  if (p) {
    if (p->struct_size != sizeof(csngf_params)) return fail(CSNGF_E_INVALID_ARG, "params.struct_size mismatch");
    prm = *p;
  }
  int rc = check_dims(dA, "A");
  if (rc) return rc;
  rc = check_dims(dB, "B");
  if (rc) return rc;
  if (!(prm.eps > 0.f) || !std::isfinite(prm.eps)) return fail(CSNGF_E_INVALID_ARG, "eps must be finite and > 0");
  if (!(prm.gamma >= 0.0 && prm.gamma <= 1.0)) return fail(CSNGF_E_INVALID_ARG, "gamma must lie in [0, 1]");
  if (prm.batch < 0 || prm.batch > 255)   // (the final pass's work list packs the slot in 8 bits)
    return fail(CSNGF_E_INVALID_ARG, "batch must lie in [0, 255]");
  if (prm.flags & ~(CSNGF_DEVICE_PTRS | CSNGF_UNSQUARED | CSNGF_GRAPHS | CSNGF_FP64))
    return fail(CSNGF_E_INVALID_ARG, "unknown flag bits");
  if (prm.slices < 0 || prm.slices > 64) return fail(CSNGF_E_INVALID_ARG, "slices must lie in [0, 64]");
  if (prm.final_groups < 0 || prm.final_groups > 65535)
    return fail(CSNGF_E_INVALID_ARG, "final_groups must lie in [0, 65535]");
  if (prm.reserved != 0) return fail(CSNGF_E_INVALID_ARG, "params.reserved must be 0");
  const int nA[3] = {dA.nx, dA.ny, dA.nz}, nB[3] = {dB.nx, dB.ny, dB.nz};
  int P[3];
  for (int i = 0; i < 3; ++i) {
    const int need = nA[i] + nB[i] - 1;
    if (prm.pad[i] == 0) {
      P[i] = auto_pad(need);
      if (P[i] < 0) return fail(CSNGF_E_UNSUPPORTED, "no supported FFT size >= n_A + n_B - 1 (max 512)");
    } else {
      if (prm.pad[i] < need) return fail(CSNGF_E_INVALID_ARG, "pad smaller than n_A + n_B - 1");
      if (!supported(prm.pad[i])) return fail(CSNGF_E_UNSUPPORTED, "pad length not supported by the FFT");
      P[i] = prm.pad[i];
    }
  }
  const size_t nvA = (size_t)dA.nx * dA.ny * dA.nz;
  if (!(prm.flags & CSNGF_DEVICE_PTRS) && !all_finite(A, nvA))
    return fail(CSNGF_E_INVALID_ARG, "fixed volume A has a non-finite value");
  rc = check_device();
  if (rc) return rc;

  csngf_ctx* c = new csngf_ctx();
  auto bail = [&](int code) {
    std::string keep = g_err;
    release(c);
    g_err = keep;
    return code;
  };
  HIPCHK(hipGetDevice(&c->dev));
  if (hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess)
    return bail(hip_fail(hipGetLastError(), "hipStreamCreateWithFlags"));
  c->stream = c->own_stream;
  for (int i = 0; i < 3; ++i) {
    c->nA[i] = nA[i];
    c->nB[i] = nB[i];
    c->P[i] = P[i];
    c->Wd[i] = nA[i] + nB[i] - 1;
  }
  c->eps = prm.eps;
  c->gamma = prm.gamma;
  if (prm.slices) c->slices = prm.slices;
  if (prm.final_groups) c->final_groups = prm.final_groups;
  c->flags = prm.flags;
  c->nf = (prm.flags & CSNGF_UNSQUARED) ? 3 : 6;
  c->H = P[0] / 2;   // bins 0 .. Px/2 - 1, bin 0 packing DC + i Nyquist
  c->Hp = (c->H + kTileW - 1) / kTileW * kTileW;
  c->tiles = (c->H + kTileW - 1) / kTileW;
  factor_plan(P[0], c->plx);
  factor_plan(P[1], c->ply);
  factor_plan(P[2], c->plz);
  c->masked = maskA != nullptr;
  c->fp64 = (prm.flags & CSNGF_FP64) != 0;
  const size_t el = c->fp64 ? sizeof(double2) : sizeof(float2);   // complex element of the fields' passes
  {
    std::vector<float2> tw;
    std::vector<double2> twd;
    c->plx.tw_off = (int)tw.size();
    twiddles(P[0], tw);
    twiddles(P[0], twd);
    c->ply.tw_off = (int)tw.size();
    twiddles(P[1], tw);
    twiddles(P[1], twd);
    c->plz.tw_off = (int)tw.size();
    twiddles(P[2], tw);
    twiddles(P[2], twd);
    if ((rc = dalloc(&c->d_tw, sizeof(float2) * tw.size()))) return bail(rc);
    if (hipMemcpy(c->d_tw, tw.data(), sizeof(float2) * tw.size(), hipMemcpyHostToDevice) != hipSuccess)
      return bail(hip_fail(hipGetLastError(), "twiddle upload"));
    if (c->masked || c->fp64) {   // same offsets as the FP32 table
      if ((rc = dalloc(&c->d_twd, sizeof(double2) * twd.size()))) return bail(rc);
      if (hipMemcpy(c->d_twd, twd.data(), sizeof(double2) * twd.size(), hipMemcpyHostToDevice) != hipSuccess)
        return bail(hip_fail(hipGetLastError(), "twiddle upload"));
    }
  }
  const long long Hp = c->Hp;
  // A's eroded mask without a user mask is the box [1, n_A - 2]; with one, its count and
  // bounding box come from the eroded mask below
  c->count_a = (long long)(nA[0] - 2) * (nA[1] - 2) * (nA[2] - 2);
  for (int i = 0; i < 3; ++i) {
    c->lo[i] = 1;
    c->hi[i] = nA[i] - 2;
  }
  c->spec_bytes = (long long)el * c->nf * P[2] * P[1] * Hp;
  if ((rc = dalloc(&c->d_spec, (size_t)c->spec_bytes))) return bail(rc);
  if ((rc = dalloc(&c->d_flag, sizeof(int)))) return bail(rc);

  // ---- fixed side: fields of A, y forward, z forward + conjugate store
  {
    const float* dA_ptr = A;
    float* tmpA = nullptr;
    if (!(prm.flags & CSNGF_DEVICE_PTRS)) {
      if ((rc = dalloc(&tmpA, sizeof(float) * nvA))) return bail(rc);
      if (hipMemcpy(tmpA, A, sizeof(float) * nvA, hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(tmpA);
        return bail(hip_fail(hipGetLastError(), "upload of A"));
      }
      dA_ptr = tmpA;
    }
    uint8_t *um = nullptr, *meff = nullptr;   // user mask on the device, A's eroded mask
    const uint8_t* dmA = maskA;
    if (c->masked) {
      rc = dalloc(&meff, nvA);
      if (!rc && !(prm.flags & CSNGF_DEVICE_PTRS)) {
        rc = dalloc(&um, nvA);
        if (!rc && hipMemcpy(um, maskA, nvA, hipMemcpyHostToDevice) != hipSuccess)
          rc = hip_fail(hipGetLastError(), "upload of mask A");
        dmA = um;
      }
    }
    if (!rc && (prm.flags & CSNGF_DEVICE_PTRS)) {
      HIPCHK(hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
      hipLaunchKernelGGL(k_check_finite, dim3(1024), dim3(256), 0, c->stream, A, (long long)nvA, c->d_flag);
    }
    if (!rc)
      rc = c->fp64 ? fixed_spectra<double2>(c, dA_ptr, dmA, nA, meff) : fixed_spectra<float2>(c, dA_ptr, dmA, nA, meff);
    if (!rc && c->masked) rc = fixed_mask_spectrum(c, meff, nA);
    hipError_t se = hipStreamSynchronize(c->stream);
    if (!rc && se != hipSuccess) rc = hip_fail(se, "fixed-side precompute");
    if (tmpA) hipFree(tmpA);
    if (um) hipFree(um);
    if (meff) hipFree(meff);
    if (rc) return bail(rc);
    int bad = 0;
    if ((rc = read_flag(c, &bad))) return bail(rc);
    if (bad) return bail(fail(CSNGF_E_INVALID_ARG, "fixed volume A has a non-finite value"));
  }

  // ---- rotation workspaces
  {
    const long long nvB = (long long)nB[0] * nB[1] * nB[2];
    c->buf1_slot = std::max((long long)c->nf * nB[2] * nB[1], (long long)c->Wd[2] * P[1]) * Hp;
    c->buf2_slot = std::max((long long)c->nf * nB[2] * P[1], (long long)c->Wd[2] * c->Wd[1]) * Hp;
    // the eroded masks, or their runs (one int2 per row) when they follow from the rotations
    c->mask_slot = (std::max(nvB, 8LL * nB[1] * nB[2]) + 255) / 256 * 256;
    c->sat_slot = ((long long)(nB[0] + 1) * (nB[1] + 1) * (nB[2] + 1) + 63) / 64 * 64;
    c->flag_slot = ((long long)c->Wd[2] * (1 + c->Wd[1]) + 255) / 256 * 256;
    const int plane_bytes = (long long)nB[0] * nB[1] < 65536 ? 2 : 4;   // per voxel, as the SAT kernels use
    c->plane_slot = ((nvB * plane_bytes + 3) / 4 + 63) / 64 * 64;
    c->work_slot = (long long)c->Wd[2] * ((c->Wd[1] + 2 * kRowsC - 1) / (2 * kRowsC));
    if (c->masked) {
      c->mbuf1_slot = std::max((long long)(nB[2] - 2) * (nB[1] - 2), (long long)c->Wd[2] * P[1]) * Hp;
      c->mbuf2_slot = std::max((long long)(nB[2] - 2) * P[1], (long long)c->Wd[2] * c->Wd[1]) * Hp;
      c->ncount_slot = ((long long)c->Wd[0] * c->Wd[1] * c->Wd[2] + 63) / 64 * 64;
    }
    const long long per = (long long)el * (c->buf1_slot + c->buf2_slot) + c->mask_slot + 4 * c->sat_slot +
                          4 * c->plane_slot + c->flag_slot + 4 * c->work_slot +
                          (long long)sizeof(double2) * (c->mbuf1_slot + c->mbuf2_slot) + 4 * c->ncount_slot;
    int batch = prm.batch;
    if (batch == 0) {
      size_t fr = 0, tot = 0;
      long long budget = 8LL << 30;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess) budget = std::min<long long>(budget, (long long)(fr / 4));
      batch = (int)std::max(1LL, std::min(64LL, budget / per));
    }
    c->batch = batch;
    if ((rc = dalloc(&c->d_buf1, el * c->buf1_slot * batch))) return bail(rc);
    if ((rc = dalloc(&c->d_buf2, el * c->buf2_slot * batch))) return bail(rc);
    if ((rc = dalloc(&c->d_plane, 4 * (size_t)c->plane_slot * batch))) return bail(rc);
    if ((rc = dalloc(&c->d_work, 4 * (64 + (size_t)c->work_slot * batch)))) return bail(rc);
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_yfwd, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_zpack, hipEventDisableTiming) != hipSuccess)
      return bail(hip_fail(hipGetLastError(), "side stream"));
    if ((rc = dalloc(&c->d_mask, (size_t)c->mask_slot * batch))) return bail(rc);
    c->brick_bytes = (long long)sizeof(float) * brick_floats(nB);
    if ((rc = dalloc(&c->d_Bb, (size_t)c->brick_bytes))) return bail(rc);
    if ((rc = dalloc(&c->d_sat, 4 * (size_t)c->sat_slot * batch))) return bail(rc);
    if ((rc = dalloc(&c->d_flags, (size_t)c->flag_slot * batch))) return bail(rc);
    if ((rc = dalloc(&c->d_keys, sizeof(unsigned long long) * batch))) return bail(rc);
    if (c->masked) {
      if ((rc = dalloc(&c->d_mbuf1, sizeof(double2) * c->mbuf1_slot * batch))) return bail(rc);
      if ((rc = dalloc(&c->d_mbuf2, sizeof(double2) * c->mbuf2_slot * batch))) return bail(rc);
      if ((rc = dalloc(&c->d_ncount, 4 * (size_t)c->ncount_slot * batch))) return bail(rc);
      if ((rc = dalloc(&c->d_ones, (size_t)c->flag_slot))) return bail(rc);
      if (hipMemsetAsync(c->d_ones, 1, (size_t)c->flag_slot, c->stream) != hipSuccess)
        return bail(hip_fail(hipGetLastError(), "hipMemsetAsync"));
    }
    if ((rc = dalloc(&c->d_rowstat, 2 * sizeof(unsigned long long)))) return bail(rc);
    // (on the context's non-blocking stream, which a null-stream memset would not order)
    if (hipMemsetAsync(c->d_rowstat, 0, 2 * sizeof(unsigned long long), c->stream) != hipSuccess)
      return bail(hip_fail(hipGetLastError(), "hipMemsetAsync"));
    if (prm.flags & CSNGF_GRAPHS) {
      if ((rc = dalloc(&c->d_rot_stage, sizeof(int) * 9 * (size_t)batch))) return bail(rc);
      if ((rc = dalloc(&c->d_res_stage, sizeof(RotResultDev) * (size_t)batch))) return bail(rc);
    }
    if (hipEventCreateWithFlags(&c->done_ev, hipEventDisableTiming) != hipSuccess)
      return bail(hip_fail(hipGetLastError(), "hipEventCreate"));
    if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(hip_fail(hipGetLastError(), "hipStreamSynchronize"));
    c->workspace_bytes = per * batch;
  }
  *out = c;
  return CSNGF_OK;
}

int csngf_set_stream(csngf_ctx* c, void* s) {
  if (!c) return fail(CSNGF_E_INVALID_ARG, "ctx is NULL");
  c->stream = s ? reinterpret_cast<hipStream_t>(s) : c->own_stream;
  return CSNGF_OK;
}

int csngf_get_info(const csngf_ctx* c, csngf_info* o) {
  if (!c || !o) return fail(CSNGF_E_INVALID_ARG, "NULL argument");
  std::memset(o, 0, sizeof(*o));
  for (int i = 0; i < 3; ++i) {
    o->pad[i] = c->P[i];
    o->map_dims[i] = c->Wd[i];
  }
  o->batch = c->batch;
  o->count_a = c->count_a;
  o->spectra_bytes = c->spec_bytes + c->brick_bytes;
  o->workspace_bytes = c->workspace_bytes;
  return CSNGF_OK;
}

int csngf_evaluate_async(csngf_ctx* c, const float* B, const uint8_t* maskB, const double* R, int32_t n) {
  if (!c) return fail(CSNGF_E_INVALID_ARG, "ctx is NULL");
  if (c->pending) return fail(CSNGF_E_INVALID_ARG, "an evaluation is already in flight on this context");
  if (!B) return fail(CSNGF_E_INVALID_ARG, "moving volume B is NULL");
  if (n < 0) return fail(CSNGF_E_INVALID_ARG, "n must be >= 0");
  if (n > 0 && !R) return fail(CSNGF_E_INVALID_ARG, "rotations are NULL");
  std::vector<int> kq((size_t)n * 9);
  for (int r = 0; r < n; ++r)
    if (quantise(R + 9 * (size_t)r, &kq[9 * (size_t)r], nullptr))
      return fail(CSNGF_E_INVALID_ARG, "rotation " + std::to_string(r) + " has a non-finite entry or |R_ij| > 2");
  HIPCHK(hipSetDevice(c->dev));
  int rc;
  if (n > 0) {
    if ((rc = ensure_rot_capacity(c, n))) return rc;
    const float* dB = nullptr;
    const uint8_t* dmB = nullptr;
    if ((rc = stage_moving(c, B, maskB, &dB, &dmB))) return rc;
    std::memcpy(c->h_rot, kq.data(), sizeof(int) * 9 * (size_t)n);
    HIPCHK(hipMemcpyAsync(c->d_rot, c->h_rot, sizeof(int) * 9 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    const bool graphs = (c->flags & CSNGF_GRAPHS) && !c->prof;
    for (int base = 0; base < n; base += c->batch) {
      const int m = std::min(c->batch, n - base);
      if (graphs && m == c->batch)
        rc = run_graph_batch(c, dB, dmB, base);
      else
        rc = run_batch(c, dB, dmB, c->d_rot + 9 * (size_t)base, m, c->d_res + base, nullptr, nullptr);
      if (rc) return rc;
    }
    HIPCHK(hipMemcpyAsync(c->h_res, c->d_res, sizeof(RotResultDev) * (size_t)n, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(hipEventRecord(c->done_ev, c->stream));
  c->pending = true;
  c->pend_n = n;
  c->pend_kq.swap(kq);
  return CSNGF_OK;
}

int csngf_query(csngf_ctx* c) {
  if (!c) return fail(CSNGF_E_INVALID_ARG, "ctx is NULL");
  if (!c->pending) return 1;
  const hipError_t e = hipEventQuery(c->done_ev);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  return hip_fail(e, "hipEventQuery");
}

int csngf_wait(csngf_ctx* c, csngf_rot_result* per_rot, csngf_best* best) {
  if (!c) return fail(CSNGF_E_INVALID_ARG, "ctx is NULL");
  if (!c->pending) return fail(CSNGF_E_INVALID_ARG, "no evaluation in flight on this context");
  c->pending = false;
  HIPCHK(hipEventSynchronize(c->done_ev));
  const int n = c->pend_n;
  int rc, bad = 0;
  if (n > 0 && (rc = read_flag(c, &bad))) return rc;
  if (bad) return fail(CSNGF_E_INVALID_ARG, "moving volume B has a non-finite value");
  int bi = -1;
  for (int r = 0; r < n; ++r) {
    const RotResultDev& x = c->h_res[r];
    if (x.valid && (bi < 0 || x.score > c->h_res[bi].score)) bi = r;
  }
  if (per_rot && n > 0) std::memcpy(per_rot, c->h_res, sizeof(csngf_rot_result) * (size_t)n);
  if (best) {
    std::memset(best, 0, sizeof(*best));
    best->rot_index = bi;
    if (bi < 0) {
      best->score = -INFINITY;
    } else {
      const RotResultDev& x = c->h_res[bi];
      best->score = x.score;
      for (int i = 0; i < 3; ++i) best->shift[i] = x.shift[i];
      best->overlap = x.overlap;
      for (int i = 0; i < 9; ++i) best->R[i] = c->pend_kq[9 * (size_t)bi + i] / 65536.0;
    }
  }
  if (bi < 0 && n > 0)
    return fail(CSNGF_E_NO_VALID_SHIFT, "no displacement meets the minimum overlap for any rotation");
  return CSNGF_OK;
}

int csngf_evaluate(csngf_ctx* c, const float* B, const uint8_t* maskB, const double* R, int32_t n,
                   csngf_rot_result* per_rot, csngf_best* best) {
  int rc = csngf_evaluate_async(c, B, maskB, R, n);
  if (rc) return rc;
  return csngf_wait(c, per_rot, best);
}

int csngf_evaluate_map(csngf_ctx* c, const float* B, const uint8_t* maskB, const double* R9, float* C,
                       int64_t* N) {
  if (!c) return fail(CSNGF_E_INVALID_ARG, "ctx is NULL");
  if (c->pending) return fail(CSNGF_E_INVALID_ARG, "an evaluation is in flight on this context");
  if (!B || !R9 || !C) return fail(CSNGF_E_INVALID_ARG, "NULL argument");
  int kq[9];
  if (quantise(R9, kq, nullptr)) return fail(CSNGF_E_INVALID_ARG, "rotation has a non-finite entry or |R_ij| > 2");
  HIPCHK(hipSetDevice(c->dev));
  int rc = ensure_rot_capacity(c, 1);
  if (rc) return rc;
  const float* dB = nullptr;
  const uint8_t* dmB = nullptr;
  if ((rc = stage_moving(c, B, maskB, &dB, &dmB))) return rc;
  const long long nmap = (long long)c->Wd[0] * c->Wd[1] * c->Wd[2];
  float* dC = C;
  long long* dN = reinterpret_cast<long long*>(N);
  float* tC = nullptr;
  long long* tN = nullptr;
  const bool host = !(c->flags & CSNGF_DEVICE_PTRS);
  if (host) {
    if ((rc = dalloc(&tC, sizeof(float) * nmap))) return rc;
    dC = tC;
    if (N) {
      if ((rc = dalloc(&tN, sizeof(long long) * nmap))) {
        hipFree(tC);
        return rc;
      }
      dN = tN;
    }
  }
  std::memcpy(c->h_rot, kq, sizeof(kq));
  auto cleanup = [&]() {
    if (tC) hipFree(tC);
    if (tN) hipFree(tN);
  };
  if (hipMemcpyAsync(c->d_rot, c->h_rot, sizeof(kq), hipMemcpyHostToDevice, c->stream) != hipSuccess) {
    cleanup();
    return hip_fail(hipGetLastError(), "rotation upload");
  }
  rc = run_batch(c, dB, dmB, c->d_rot, 1, c->d_res, dC, dN);
  hipError_t se = hipStreamSynchronize(c->stream);
  if (!rc && se != hipSuccess) rc = hip_fail(se, "csngf_evaluate_map");
  int bad = 0;
  if (!rc) rc = read_flag(c, &bad);
  if (!rc && bad) rc = fail(CSNGF_E_INVALID_ARG, "moving volume B has a non-finite value");
  if (!rc && host) {
    if (hipMemcpy(C, dC, sizeof(float) * nmap, hipMemcpyDeviceToHost) != hipSuccess)
      rc = hip_fail(hipGetLastError(), "map download");
    if (!rc && N && hipMemcpy(N, dN, sizeof(long long) * nmap, hipMemcpyDeviceToHost) != hipSuccess)
      rc = hip_fail(hipGetLastError(), "overlap download");
  }
  cleanup();
  return rc;
}

int csngf_destroy(csngf_ctx* c) {
  if (!c) return fail(CSNGF_E_INVALID_ARG, "ctx is NULL");
  release(c);
  return CSNGF_OK;
}

}  // extern "C"

namespace {

// Normalised Gaussian taps of csngf_smooth_downsample, computed in double and rounded once.
void blur_taps(float sigma, BlurTaps* t, int* K) {
  const int k = sigma > 0.f ? (int)(4.0 * sigma + 0.5) : 0;
  std::vector<double> wd(2 * k + 1);
  double sum = 0;
  for (int j = -k; j <= k; ++j) {
    wd[j + k] = k ? std::exp(-(double)j * j / (2.0 * (double)sigma * sigma)) : 1.0;
    sum += wd[j + k];
  }
  std::memset(t, 0, sizeof(*t));
  for (int j = 0; j <= 2 * k; ++j) t->w[j] = (float)(wd[j] / sum);
  *K = k;
}

// The three separable passes: x keeps m0 of n0 columns (din -> t1), y m1 of n1 rows (t1 -> t2),
// z m2 of n2 slices (t2 -> dout).  t1 holds m0 n1 n2 floats, t2 m0 m1 n2.
hipError_t launch_pyramid(const float* din, float* t1, float* t2, float* dout, const int* n, const int* m, int factor,
                          const BlurTaps& taps, int K, hipStream_t s) {
  auto blur = [&](const float* a, float* b, int outer, int len, int inner, int mm) {
    const long long total = (long long)outer * mm * inner;
    hipLaunchKernelGGL(k_blur_axis, dim3((unsigned)((total + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, a, b,
                       outer, len, inner, mm, factor, taps, K);
  };
  blur(din, t1, n[2] * n[1], n[0], 1, m[0]);          // along x
  blur(t1, t2, n[2], n[1], m[0], m[1]);               // along y
  blur(t2, dout, 1, n[2], m[1] * m[0], m[2]);         // along z
  return hipGetLastError();
}

int pyramid_args(const float* vol, csngf_dims d, float sigma, int32_t factor, csngf_dims* out_dims, int* n, int* m) {
  if (!vol || !out_dims) return fail(CSNGF_E_INVALID_ARG, "NULL argument");
  if (d.nx < 1 || d.ny < 1 || d.nz < 1) return fail(CSNGF_E_INVALID_ARG, "extents must be >= 1");
  if (factor < 1) return fail(CSNGF_E_INVALID_ARG, "factor must be >= 1");
  if (!(sigma >= 0.f && sigma <= 64.f)) return fail(CSNGF_E_INVALID_ARG, "sigma must lie in [0, 64]");
  n[0] = d.nx;
  n[1] = d.ny;
  n[2] = d.nz;
  for (int i = 0; i < 3; ++i) m[i] = (n[i] + factor - 1) / factor;
  *out_dims = csngf_dims{m[0], m[1], m[2]};
  return CSNGF_OK;
}

// Scratch of csngf_smooth_downsample_noalloc: the two intermediate volumes of the separable
// blur.  Each device the library runs on holds its own copy until the process ends.  In host
// code the name stands for the host-side shadow, not a device address: kernels get the
// address from scratch_on_current_device().
constexpr size_t kScratchFloats = CSNGF_NOALLOC_SCRATCH_BYTES / sizeof(float);
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The device address of scratch on the current device, looked up once per device.
int scratch_on_current_device(float** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CSNGF_E_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return CSNGF_OK;
}

}  // namespace

extern "C" {

int csngf_smooth_downsample(const float* vol, csngf_dims d, float sigma, int32_t factor, float* out,
                            csngf_dims* out_dims, uint32_t flags, void* stream) {
  int n[3], m[3];
  int rc = pyramid_args(vol, d, sigma, factor, out_dims, n, m);
  if (rc) return rc;
  if (flags & ~CSNGF_DEVICE_PTRS) return fail(CSNGF_E_INVALID_ARG, "unknown flag bits");
  if (!out) return CSNGF_OK;
  if ((rc = check_device())) return rc;
  const bool dev = flags & CSNGF_DEVICE_PTRS;
  const size_t nv = (size_t)n[0] * n[1] * n[2], mv = (size_t)m[0] * m[1] * m[2];
  if (!dev && !all_finite(vol, nv)) return fail(CSNGF_E_INVALID_ARG, "non-finite volume");
  BlurTaps taps;
  int K = 0;
  blur_taps(sigma, &taps, &K);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<void*> owned;
  auto done = [&](int code) {
    (void)hipStreamSynchronize(s);
    for (void* p : owned) (void)hipFree(p);
    return code;
  };
  float *t1 = nullptr, *t2 = nullptr, *din = const_cast<float*>(vol), *dout = out;
  if ((rc = dalloc(&t1, sizeof(float) * (size_t)m[0] * n[1] * n[2]))) return done(rc);
  owned.push_back(t1);
  if ((rc = dalloc(&t2, sizeof(float) * (size_t)m[0] * m[1] * n[2]))) return done(rc);
  owned.push_back(t2);
  if (!dev) {
    if ((rc = dalloc(&din, sizeof(float) * nv))) return done(rc);
    owned.push_back(din);
    if ((rc = dalloc(&dout, sizeof(float) * mv))) return done(rc);
    owned.push_back(dout);
    if (hipMemcpyAsync(din, vol, sizeof(float) * nv, hipMemcpyHostToDevice, s) != hipSuccess)
      return done(hip_fail(hipGetLastError(), "upload"));
  }
  const hipError_t e = launch_pyramid(din, t1, t2, dout, n, m, factor, taps, K, s);
  if (e != hipSuccess) return done(hip_fail(e, "k_blur_axis"));
  if (!dev) {
    if (hipMemcpyAsync(out, dout, sizeof(float) * mv, hipMemcpyDeviceToHost, s) != hipSuccess)
      return done(hip_fail(hipGetLastError(), "download"));
  }
  return done(CSNGF_OK);
}

int csngf_smooth_downsample_noalloc(const float* vol, csngf_dims d, float sigma, int32_t factor, float* out,
                                    csngf_dims* out_dims, void* stream) {
  int n[3], m[3];
  int rc = pyramid_args(vol, d, sigma, factor, out_dims, n, m);
  if (rc) return rc;
  if (!out) return CSNGF_OK;
  const unsigned long long need1 = (unsigned long long)m[0] * n[1] * n[2];
  const unsigned long long need2 = (unsigned long long)m[0] * m[1] * n[2];
  // each intermediate starts on a 256-byte boundary of the scratch array
  const unsigned long long off2 = (need1 + 63) / 64 * 64;
  if (off2 + need2 > kScratchFloats)
    return fail(CSNGF_E_UNSUPPORTED, "volume too large for the allocation-free pyramid: its intermediates need " +
                                          std::to_string(4 * (off2 + need2)) + " bytes of the " +
                                          std::to_string(CSNGF_NOALLOC_SCRATCH_BYTES) + "-byte scratch");
  if ((rc = check_device())) return rc;
  float* base = nullptr;
  if ((rc = scratch_on_current_device(&base))) return rc;
  BlurTaps taps;
  int K = 0;
  blur_taps(sigma, &taps, &K);
  const hipError_t e = launch_pyramid(vol, base, base + off2, out, n, m, factor, taps, K,
                                      reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "k_blur_axis");
  return CSNGF_OK;
}

// ---------------------------------------------------------------------------- footprint
extern "C" int csngf_footprint(csngf_dims dA, csngf_dims dB, const csngf_params* p, int64_t* spectra_bytes,
                               int64_t* slot_bytes, int32_t* pad_out) {
  csngf_params prm;
  csngf_default_params(&prm);
  if (p) {
    if (p->struct_size != sizeof(csngf_params)) return fail(CSNGF_E_INVALID_ARG, "params.struct_size mismatch");
    prm = *p;
  }
  int rc = check_dims(dA, "A");
  if (rc) return rc;
  if ((rc = check_dims(dB, "B"))) return rc;
  const int nA[3] = {dA.nx, dA.ny, dA.nz}, nB[3] = {dB.nx, dB.ny, dB.nz};
  int P[3], Wd[3];
  for (int i = 0; i < 3; ++i) {
    const int need = nA[i] + nB[i] - 1;
    P[i] = prm.pad[i] ? prm.pad[i] : auto_pad(need);
    if (P[i] < need || !supported(P[i])) return fail(CSNGF_E_UNSUPPORTED, "FFT size not available");
    Wd[i] = need;
  }
  const int nf = (prm.flags & CSNGF_UNSQUARED) ? 3 : 6;
  const long long el = (prm.flags & CSNGF_FP64) ? (long long)sizeof(double2) : (long long)sizeof(float2);
  const long long H = P[0] / 2, Hp = (H + kTileW - 1) / kTileW * kTileW;
  const long long nvB = (long long)nB[0] * nB[1] * nB[2];
  const long long buf1 = std::max((long long)nf * nB[2] * nB[1], (long long)Wd[2] * P[1]) * Hp;
  const long long buf2 = std::max((long long)nf * nB[2] * P[1], (long long)Wd[2] * Wd[1]) * Hp;
  const int plane_bytes = (long long)nB[0] * nB[1] < 65536 ? 2 : 4;
  const long long per = el * (buf1 + buf2) + (std::max(nvB, 8LL * nB[1] * nB[2]) + 255) / 256 * 256 +
                        4 * (((long long)(nB[0] + 1) * (nB[1] + 1) * (nB[2] + 1) + 63) / 64 * 64) +
                        4 * (((nvB * plane_bytes + 3) / 4 + 63) / 64 * 64) +
                        ((long long)Wd[2] * (1 + Wd[1]) + 255) / 256 * 256 +
                        4LL * Wd[2] * ((Wd[1] + 2 * kRowsC - 1) / (2 * kRowsC));
  if (spectra_bytes) *spectra_bytes = el * nf * P[2] * P[1] * Hp + (long long)sizeof(float) * brick_floats(nB);
  if (slot_bytes) *slot_bytes = per;
  if (pad_out)
    for (int i = 0; i < 3; ++i) pad_out[i] = P[i];
  return CSNGF_OK;
}

// ---------------------------------------------------------------------------- autotuner
namespace {

// Deterministic probe rotations: normalised Gaussian quaternions from a fixed seed.
std::vector<double> probe_rotations(int n) {
  std::mt19937 gen(20211019u);
  std::normal_distribution<double> nd(0.0, 1.0);
  std::vector<double> R((size_t)n * 9);
  for (int i = 0; i < n; ++i) {
    double w = nd(gen), x = nd(gen), y = nd(gen), z = nd(gen);
    const double s = 1.0 / std::sqrt(w * w + x * x + y * y + z * z);
    w *= s; x *= s; y *= s; z *= s;
    double* r = &R[9 * (size_t)i];
    r[0] = 1 - 2 * (y * y + z * z); r[1] = 2 * (x * y - w * z);     r[2] = 2 * (x * z + w * y);
    r[3] = 2 * (x * y + w * z);     r[4] = 1 - 2 * (x * x + z * z); r[5] = 2 * (y * z - w * x);
    r[6] = 2 * (x * z - w * y);     r[7] = 2 * (y * z + w * x);     r[8] = 1 - 2 * (x * x + y * y);
  }
  return R;
}
}  // namespace

extern "C" int csngf_autotune(const float* A, csngf_dims dA, const float* B, csngf_dims dB, const csngf_params* base,
                              int32_t n_probe, csngf_params* best, double* best_rate) {
  if (!A || !B || !best) return fail(CSNGF_E_INVALID_ARG, "NULL argument");
  if (n_probe < 1) return fail(CSNGF_E_INVALID_ARG, "n_probe must be >= 1");
  csngf_params prm;
  csngf_default_params(&prm);
  if (base) {
    if (base->struct_size != sizeof(csngf_params)) return fail(CSNGF_E_INVALID_ARG, "params.struct_size mismatch");
    prm = *base;
  }
  const int nA[3] = {dA.nx, dA.ny, dA.nz}, nB[3] = {dB.nx, dB.ny, dB.nz};
  std::vector<int> cand[3];
  for (int i = 0; i < 3; ++i) {
    const int need = nA[i] + nB[i] - 1;
    const int s0 = smallest_supported_at_least(need);
    if (s0 < 0) return fail(CSNGF_E_UNSUPPORTED, "no supported FFT size >= n_A + n_B - 1");
    cand[i].push_back(s0);
    // and the next length with a compile-time plan within 1.5x: a longer length of cheaper
    // radices (say 128 = 8 4 4 for 110 = 11 5 2) can be the faster transform
    for (int L = s0 + 1; L <= kMaxLen && L <= need + need / 2; ++L)
      if (fast_length(L)) {
        cand[i].push_back(L);
        break;
      }
  }
  const std::vector<double> R = probe_rotations(n_probe);
  std::vector<csngf_rot_result> per((size_t)n_probe);
  double best_r = -1.0;
  csngf_params best_p = prm;
  auto probe = [&](csngf_params q, int* used_batch) -> double {
    csngf_ctx* ctx = nullptr;
    if (csngf_create(A, dA, nullptr, dB, &q, &ctx) != CSNGF_OK) return -1.0;
    *used_batch = ctx->batch;
    double rate = -1.0;
    int rc = csngf_evaluate(ctx, B, nullptr, R.data(), n_probe, per.data(), nullptr);
    if (rc == CSNGF_OK || rc == CSNGF_E_NO_VALID_SHIFT) {
      const auto t0 = std::chrono::steady_clock::now();
      rc = csngf_evaluate(ctx, B, nullptr, R.data(), n_probe, per.data(), nullptr);
      const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (rc == CSNGF_OK || rc == CSNGF_E_NO_VALID_SHIFT) rate = n_probe / dt;
    }
    csngf_destroy(ctx);
    return rate;
  };
  // FFT sizes with the automatic slot count, then half and double the slots at the best size
  for (int px : cand[0])
    for (int py : cand[1])
      for (int pz : cand[2]) {
        csngf_params q = prm;
        q.pad[0] = px;
        q.pad[1] = py;
        q.pad[2] = pz;
        q.batch = 0;
        int b0 = 0;
        const double r0 = probe(q, &b0);
        if (r0 > best_r) { best_r = r0; best_p = q; best_p.batch = b0; }
      }
  if (best_r <= 0) return fail(CSNGF_E_DEVICE, "no candidate configuration could be evaluated");
  {
    const csngf_params base_b = best_p;
    for (int b : {base_b.batch / 2, base_b.batch * 2}) {
      if (b < 1 || b > 64) continue;
      csngf_params q = base_b;
      q.batch = b;
      int bu = 0;
      const double r = probe(q, &bu);
      if (r > best_r) { best_r = r; best_p = q; }
    }
  }
  // launch shapes, one knob at a time from the best FFT size and slot count
  {
    const csngf_params base_p = best_p;
    for (int sl : {4, 16}) {
      csngf_params q = base_p;
      q.slices = sl;
      int bu = 0;
      const double r = probe(q, &bu);
      if (r > best_r) { best_r = r; best_p = q; }
    }
    const csngf_params base_f = best_p;
    for (int fg : {2048, 4096, 16384}) {
      csngf_params q = base_f;
      q.final_groups = fg;
      int bu = 0;
      const double r = probe(q, &bu);
      if (r > best_r) { best_r = r; best_p = q; }
    }
  }
  if (best_p.slices == 0) best_p.slices = kSlicesX;
  if (best_p.final_groups == 0) best_p.final_groups = kFinalGroups;
  *best = best_p;
  if (best_rate) *best_rate = best_r;
  return CSNGF_OK;
}

// ---------------------------------------------------------------------------- debug / profile
int csngf_debug_fft(const void* in, void* out, int32_t L, int32_t batch, int32_t inverse, void* stream) {
  if (!in || !out || batch < 0) return fail(CSNGF_E_INVALID_ARG, "bad argument");
  if (!supported(L)) return fail(CSNGF_E_UNSUPPORTED, "FFT length not supported");
  int rc = check_device();
  if (rc) return rc;
  if (batch == 0) return CSNGF_OK;
  FftPlan pl;
  factor_plan(L, pl);
  pl.tw_off = 0;
  std::vector<float2> tw;
  twiddles(L, tw);
  float2* dtw = nullptr;
  if ((rc = dalloc(&dtw, sizeof(float2) * L))) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(dtw, tw.data(), sizeof(float2) * L, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    const dim3 grid((batch + kTileW - 1) / kTileW);
    const size_t lds = lds_pencil(L);
    with_len(L, [&](auto lc) {
      constexpr int LC = decltype(lc)::value;
      if (inverse)
        hipLaunchKernelGGL((k_debug_fft<true, LC>), grid, dim3(kThreadsP<true>), lds, s, (const float2*)in, (float2*)out,
                           batch, pl, dtw);
      else
        hipLaunchKernelGGL((k_debug_fft<false, LC>), grid, dim3(kThreadsP<false>), lds, s, (const float2*)in, (float2*)out,
                           batch, pl, dtw);
    });
    e = hipGetLastError();
  }
  hipError_t se = hipStreamSynchronize(s);
  hipFree(dtw);
  if (e != hipSuccess) return hip_fail(e, "k_debug_fft");
  if (se != hipSuccess) return hip_fail(se, "k_debug_fft sync");
  return CSNGF_OK;
}

int csngf_debug_fields(const float* vol, const uint8_t* vmask, csngf_dims d, const double* R9, float eps, int32_t Px,
                       float* prod6, uint8_t* mask, uint32_t flags) {
  if (!vol || !prod6 || !mask) return fail(CSNGF_E_INVALID_ARG, "NULL argument");
  int rc = check_dims(d, "volume");
  if (rc) return rc;
  if (!(eps > 0.f)) return fail(CSNGF_E_INVALID_ARG, "eps must be > 0");
  if (Px == 0) Px = smallest_supported_at_least(2 * d.nx - 1);
  if (Px < d.nx || !supported(Px)) return fail(CSNGF_E_UNSUPPORTED, "Px not supported");
  int kq[9];
  if (R9 && quantise(R9, kq, nullptr)) return fail(CSNGF_E_INVALID_ARG, "bad rotation");
  if ((rc = check_device())) return rc;
  const bool dev = flags & CSNGF_DEVICE_PTRS;
  const size_t nv = (size_t)d.nx * d.ny * d.nz;
  if (!dev && !all_finite(vol, nv)) return fail(CSNGF_E_INVALID_ARG, "non-finite volume");
  csngf_ctx tmp;
  tmp.stream = nullptr;
  tmp.eps = eps;
  tmp.nf = (flags & CSNGF_UNSQUARED) ? 3 : 6;
  factor_plan(Px, tmp.plx);
  tmp.plx.tw_off = 0;
  tmp.H = Px / 2;
  tmp.Hp = (tmp.H + kTileW - 1) / kTileW * kTileW;
  std::vector<float2> tw;
  twiddles(Px, tw);
  float* dvol = const_cast<float*>(vol);
  uint8_t* dvm = const_cast<uint8_t*>(vmask);
  float* dprod = prod6;
  uint8_t* dmask = mask;
  float2* x1 = nullptr;
  int* drot = nullptr;
  std::vector<void*> owned;
  auto done = [&](int code) {
    hipDeviceSynchronize();
    for (void* p : owned) hipFree(p);
    if (tmp.d_tw) hipFree(tmp.d_tw);
    tmp.d_tw = nullptr;
    return code;
  };
  const int n3[3] = {d.nx, d.ny, d.nz};
  if ((rc = dalloc(&tmp.d_tw, sizeof(float2) * Px))) return done(rc);
  if ((rc = dalloc(&x1, sizeof(float2) * tmp.nf * (size_t)d.nz * d.ny * tmp.Hp))) return done(rc);
  owned.push_back(x1);
  if ((rc = dalloc(&drot, sizeof(kq)))) return done(rc);
  owned.push_back(drot);
  if (hipMemcpy(tmp.d_tw, tw.data(), sizeof(float2) * Px, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(drot, kq, sizeof(kq), hipMemcpyHostToDevice) != hipSuccess)
    return done(hip_fail(hipGetLastError(), "upload"));
  if (!dev) {
    if ((rc = dalloc(&dvol, sizeof(float) * nv))) return done(rc);
    owned.push_back(dvol);
    if (hipMemcpy(dvol, vol, sizeof(float) * nv, hipMemcpyHostToDevice) != hipSuccess)
      return done(hip_fail(hipGetLastError(), "upload"));
    if (vmask) {
      if ((rc = dalloc(&dvm, nv))) return done(rc);
      owned.push_back(dvm);
      if (hipMemcpy(dvm, vmask, nv, hipMemcpyHostToDevice) != hipSuccess)
        return done(hip_fail(hipGetLastError(), "upload"));
    }
    if ((rc = dalloc(&dprod, sizeof(float) * tmp.nf * nv))) return done(rc);
    owned.push_back(dprod);
    if ((rc = dalloc(&dmask, nv))) return done(rc);
    owned.push_back(dmask);
  }
  float* gvol = dvol;   // the moving side gathers from a brick copy
  if (R9) {
    if ((rc = dalloc(&gvol, sizeof(float) * brick_floats(n3)))) return done(rc);
    owned.push_back(gvol);
    if ((rc = launch_brick(nullptr, dvol, n3, gvol))) return done(rc);
  }
  rc = launch_fields(&tmp, R9 != nullptr, gvol, dvm, n3, drot, x1, 0, dmask, 0, dprod, 1);
  if (rc) return done(rc);
  if (hipDeviceSynchronize() != hipSuccess) return done(hip_fail(hipGetLastError(), "k_fields_x"));
  if (!dev) {
    if (hipMemcpy(prod6, dprod, sizeof(float) * tmp.nf * nv, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(mask, dmask, nv, hipMemcpyDeviceToHost) != hipSuccess)
      return done(hip_fail(hipGetLastError(), "download"));
  }
  return done(CSNGF_OK);
}

int csngf_profile_enable(csngf_ctx* c, int32_t enable) {
  if (!c) return fail(CSNGF_E_INVALID_ARG, "ctx is NULL");
  c->prof = enable != 0;
  return CSNGF_OK;
}

int csngf_profile_read(csngf_ctx* c, csngf_kernel_stat* out, int32_t max, int32_t* count) {
  if (!c) return fail(CSNGF_E_INVALID_ARG, "ctx is NULL");
  HIPCHK(hipStreamSynchronize(c->stream));
  prof_fold(c);
  if (count) *count = KT_COUNT;
  for (int i = 0; out && i < KT_COUNT && i < max; ++i) {
    std::memset(&out[i], 0, sizeof(out[i]));
    std::snprintf(out[i].name, sizeof(out[i].name), "%s", kTypeName[i]);
    out[i].launches = c->stat_launches[i];
    out[i].total_ms = c->stat_ms[i];
  }
  return CSNGF_OK;
}

int csngf_profile_reset(csngf_ctx* c) {
  if (!c) return fail(CSNGF_E_INVALID_ARG, "ctx is NULL");
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipStreamSynchronize(c->side));
  prof_fold(c);
  for (int i = 0; i < KT_COUNT; ++i) {
    c->stat_launches[i] = 0;
    c->stat_ms[i] = 0;
  }
  HIPCHK(hipMemsetAsync(c->d_rowstat, 0, 2 * sizeof(unsigned long long), c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->stat_rotations = 0;
  return CSNGF_OK;
}

int csngf_profile_rows(csngf_ctx* c, int64_t* z_rows, int64_t* rows, int64_t* rotations) {
  if (!c) return fail(CSNGF_E_INVALID_ARG, "ctx is NULL");
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipStreamSynchronize(c->side));
  unsigned long long h[2] = {0, 0};
  HIPCHK(hipMemcpy(h, c->d_rowstat, sizeof(h), hipMemcpyDeviceToHost));
  if (z_rows) *z_rows = (int64_t)h[0];
  if (rows) *rows = (int64_t)h[1];
  if (rotations) *rotations = c->stat_rotations;
  return CSNGF_OK;
}

}  // extern "C"
