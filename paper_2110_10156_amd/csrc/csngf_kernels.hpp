// HIP kernels of the CSNGF hot path (gfx950).
//
// Data flow for one rotation slot (H = Px/2 stored half-spectrum bins along x, row pitch Hp):
//   k_fields_x   B -> resample -> NGF -> mask -> 6 products -> x R2C    X1 [6][nz-2][ny-2][Hp]
//   k_mask_runs, k_sat_*   eroded mask of B^ (runs of x per row from the rotation, or the
//                field stage's mask bytes) -> zero-bordered 3-D summed-area table (exact overlaps)
//   k_pencil<F>  y forward, ny-2 nonzero rows -> Py                      X2 [6][nz-2][Py][Hp]
//   k_zpass      per field: z forward (nz-2 nonzero -> Pz), multiply by A's conjugate spectrum,
//                sum over fields; then z inverse of the sum              Y3 [Wz][Py][Hp]
//   k_pencil<I>  y inverse, kept rows = displacement range               Y4 [Wz][Wy][Hp]
//   k_final_x    x C2R -> S(chi); N(chi) from the SAT; gamma; C = S/N; per-slot argmax key
// Fixed side (once per context): k_fields_x<direct>, k_pencil<F>, k_zstore (conjugate,
// cross-term weight 2, 1/(Px Py Pz)).
//
// Packed DC/Nyquist column.  The x R2C of a real row has Px/2 + 1 bins, of which bin 0 (DC)
// and bin Px/2 (Nyquist) are real.  Bin 0 carries both, as DC + i Nyquist, so a row holds
// Px/2 bins and the pencil passes run Px/2 / 16 tiles instead of one more, nearly empty one.
// Along the pencil passes that column (x-bin 0, the first pencil of tile 0) is kept as:
//   after the y forward, rows ky in (0, Py/2) hold the DC plane's D(ky), rows Py - ky its
//   Nyquist plane's N(ky) (both planes are FFTs of real data, so D(-ky) = conj D(ky) and
//   likewise N); rows 0 and Py/2 hold D + i N, both real there;
//   A's spectra and the z pass keep the same rows; at ky = 0 and Py/2 the same split is made
//   once more along kz (k_zstore, the packed branch of k_zpass), so the products summed there
//   are again D-plane + i Nyquist-plane, whose z inverse is real + i real;
//   the y inverse rebuilds S_D(ky) + i S_N(ky) from rows ky and Py - ky, so the x C2R finds
//   DC + i Nyquist of every displacement row in bin 0.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csngf_fft.hpp"

namespace csngf {

constexpr int kThreads = 256;  // workgroup size of the small kernels
constexpr int kTileW = 16;     // adjacent x-bins per pencil tile in the z pass (and row pitch unit)
// Workgroup sizes and y tile widths of the FFT passes.  LDS, not registers, limits how many
// workgroups a CU holds in these passes, so a larger workgroup raises the resident waves.
// Defaults are the fastest measured on a 176x176x110 pair (FFT 352x352x220); each can be
// overridden at build time (-DCSNGF_TF=... and so on) for tuning.
#ifndef CSNGF_TF
#define CSNGF_TF 512
#endif
#ifndef CSNGF_TPF
#define CSNGF_TPF 512   // y forward: 0.087 -> 0.084 ms per rotation against 256 (more waves in flight)
#endif
#ifndef CSNGF_TPI
#define CSNGF_TPI 512
#endif
#ifndef CSNGF_TZ
#define CSNGF_TZ 512
#endif
#ifndef CSNGF_TC
#define CSNGF_TC 256
#endif
#ifndef CSNGF_WPF
#define CSNGF_WPF 16
#endif
#ifndef CSNGF_WPI
#define CSNGF_WPI 16
#endif
constexpr int kThreadsF = CSNGF_TF;  // field stage (x pass)
constexpr int kThreadsZ = CSNGF_TZ;  // z pass
constexpr int kThreadsC = CSNGF_TC;  // final x pass (C2R, normalisation, argmax)
static_assert(kThreadsC % 64 == 0 && (kThreadsC <= 256 || kThreadsC % 256 == 0), "the final pass maps min(T, 256) threads per D row");
template <bool INV>
constexpr int kThreadsP = INV ? CSNGF_TPI : CSNGF_TPF;  // y pencil passes (forward, inverse)
template <bool INV>
constexpr int kTileP = INV ? CSNGF_WPI : CSNGF_WPF;     // x-bins per y pencil tile
static_assert(kTileW % CSNGF_WPF == 0 && kTileW % CSNGF_WPI == 0, "y tiles must divide the row pitch unit");
constexpr int kRowsX = 8;    // rows per workgroup in the field stage
// halo samples per gather group in the field stage; the group loop is fully unrolled, so
// the compiler interleaves the groups' gathers itself (1 measured fastest, 4 about 3% slower)
#ifndef CSNGF_HU
#define CSNGF_HU 1
#endif
#ifndef CSNGF_GBW
#define CSNGF_GBW 16
#endif
constexpr int kGatherGroup = CSNGF_HU;
constexpr int kGatherBW = CSNGF_GBW;   // columns per block of the field stage's sample-to-thread map
#ifndef CSNGF_ROWSC
#define CSNGF_ROWSC 4
#endif
constexpr int kRowsC = CSNGF_ROWSC;  // packed row pairs per workgroup in the final pass

struct RotResultDev {        // identical layout to csngf_rot_result
  float score;
  int32_t shift[3];
  long long overlap;
  int32_t valid;
  int32_t reserved;
};

__device__ __forceinline__ float lerp_exact(float a, float b, float f) {
  // a + f (b - a): returns a exactly when a == b, so constant regions stay constant
  return fmaf(f, b - a, a);
}

__device__ __forceinline__ size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

// ------------------------------------------------------------------------- buffer views
// A raw buffer resource over [base, base + bytes) with a workgroup-uniform base.  Element
// accesses take a 32-bit byte offset (one 24-bit multiply-add per element instead of 64-bit
// address arithmetic), and the hardware range check returns zero for a load, and drops a
// store, at any offset >= bytes: a predicated access passes kNoOff instead of branching.
// Every view here spans less than 2 GiB, so kNoOff is always out of range.
constexpr uint32_t kNoOff = 0x80000000u;
typedef unsigned int u32x2 __attribute__((__vector_size__(8)));
typedef unsigned int u32x4 __attribute__((__vector_size__(16)));

// Cache policy of the intermediates: every pass writes its output once, for the next pass
// to read once, so stores (bit 0) and those loads (bit 1) are non-temporal.  That keeps them
// from evicting what is reused: B's neighbourhoods during the gathers and A's spectra tiles
// in the z pass.  Measured +5% on the whole path.
#ifndef CSNGF_NT
#define CSNGF_NT 3
#endif
constexpr bool kStreamSt = (CSNGF_NT & 1) != 0;
constexpr bool kStreamLd = (CSNGF_NT & 2) != 0;
struct RView {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ RView(const void* base, long long bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000)) {}
  // (whole-object copies: a bit cast of a single vector element is miscompiled by this
  // compiler into a read of element 0)
  __device__ __forceinline__ float2 ld2(uint32_t off, uint32_t soff = 0) const {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, (int)soff, 0);
    float2 x;
    __builtin_memcpy(&x, &v, 8);
    return x;
  }
  // a float2 read once and never again (a pass's input pencils): non-temporal when kStreamLd
  __device__ __forceinline__ float2 ld2s(uint32_t off, uint32_t soff = 0) const {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, (int)soff, kStreamLd ? 2 : 0);
    float2 x;
    __builtin_memcpy(&x, &v, 8);
    return x;
  }
  __device__ __forceinline__ void st2(uint32_t off, float2 x) const {
    u32x2 v;
    __builtin_memcpy(&v, &x, 8);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)off, 0, kStreamSt ? 2 : 0);
  }
  // complex element of type V (float2 or double2); STREAM: read once (non-temporal when
  // kStreamLd), as ld2s
  template <typename V, bool STREAM>
  __device__ __forceinline__ V ldv(uint32_t off, uint32_t soff = 0) const {
    if constexpr (sizeof(V) == 8) {
      return STREAM ? ld2s(off, soff) : ld2(off, soff);
    } else {
      const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, (int)soff, (STREAM && kStreamLd) ? 2 : 0);
      V x;
      __builtin_memcpy(&x, &v, 16);
      return x;
    }
  }
  template <typename V>
  __device__ __forceinline__ void stv(uint32_t off, V x) const {
    if constexpr (sizeof(V) == 8) {
      st2(off, x);
    } else {
      u32x4 v;
      __builtin_memcpy(&v, &x, 16);
      __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)off, 0, kStreamSt ? 2 : 0);
    }
  }
  __device__ __forceinline__ unsigned ld1(uint32_t off, uint32_t soff = 0) const {
    return __builtin_amdgcn_raw_buffer_load_b8(r, (int)off, (int)soff, 0);
  }
  __device__ __forceinline__ void st1(uint32_t off, unsigned char x) const {
    __builtin_amdgcn_raw_buffer_store_b8(x, r, (int)off, 0, 0);
  }
  __device__ __forceinline__ int ldi(uint32_t off) const {
    return (int)__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
  }
  // float at byte offset off + soff (soff: a workgroup-uniform offset held in a scalar register)
  __device__ __forceinline__ float ldf(uint32_t off, uint32_t soff = 0) const {
    const unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, (int)soff, 0);
    float x;
    __builtin_memcpy(&x, &v, 4);
    return x;
  }
};

// byte offset of element (row, col) of an array of complex V with a row stride of rsb bytes
// (row < 2^24 and rsb < 2^24, offset < 2^31; rsb workgroup-uniform)
template <typename V>
__device__ __forceinline__ uint32_t offv(int row, uint32_t rsb, int col) {
  return mad24u((unsigned)row, rsb, (uint32_t)sizeof(V) * (unsigned)col);
}
// offv when ok, else kNoOff.  The offset is formed unconditionally and then selected: as a
// conditional expression around offv the compiler would branch around the multiply.
template <typename V>
__device__ __forceinline__ uint32_t offv_if(bool ok, int row, uint32_t rsb, int col) {
  const uint32_t o = offv<V>(row, rsb, col);
  return ok ? o : kNoOff;
}

// ------------------------------------------------------------------------------ B in bricks
// The moving side gathers B through a copy in bricks of 4 x 4 x 4 trilinear cells with their
// upper corners: 5 x 5 x 5 values (x fastest), brick (bx, by, bz) holding B at
// (4 bx + lx, 4 by + ly, 4 bz + lz), lx, ly, lz = 0..4, clamped to the grid.  Every cell's 8
// corners then lie in one 500-byte brick, as (x, x+1) pairs 0, 5, 25 and 30 values apart, and
// a wave's gathers over a rotated patch touch few cache lines.  nbx = ceil((nx - 1) / 4)
// bricks per axis cover the nx - 1 cells.
constexpr int kBrickVals = 125;
__host__ __device__ constexpr int brick_count(int n) { return (n + 2) / 4; }   // ceil((n - 1) / 4)

__global__ __launch_bounds__(kThreads) void k_brick(const float* __restrict__ B, int nx, int ny, int nz,
                                                    float* __restrict__ out, long long total) {
  const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (t >= total) return;
  const int nbx = brick_count(nx), nby = brick_count(ny);
  const int b = (int)(t / kBrickVals), l = (int)(t - (long long)b * kBrickVals);
  const int lz = l / 25, ly = (l - 25 * lz) / 5, lx = l - 25 * lz - 5 * ly;
  const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
  const int x = min(4 * bx + lx, nx - 1), y = min(4 * by + ly, ny - 1), z = min(4 * bz + lz, nz - 1);
  out[t] = B[((long long)z * ny + y) * nx + x];
}

// ------------------------------------------------------------------------------ x pass
// One workgroup: rows y0 .. y0+kRowsX-1 of slices z0 .. z0+tz-1 of one rotation slot,
// marching along z with a ring of 3 sampled halo planes (rows y0-1 .. y0+kRowsX) in LDS, so
// each new slice costs one new plane.  A sample that is not valid (outside the grid or the
// box, or a mask corner unset) is stored as NaN, so one NaN test on the gradient stencil
// gives the eroded mask.  Per slice: mask and NGF once per voxel into LDS; then for each of
// the 3 field pairs (xx,yy), (zz,xy), (xz,yz) the first FFT stage forms the pair's products
// (re = first field, im = second), the transform runs along x (length Px, zero padded from
// nx) and the result is split into two half spectra.
//
// HALF: nx <= Px / 2, so the transform's inputs x >= Px / 2 are known zero (first stage pruned).
// Every strided loop visits the same elements in every plane, so each thread decodes its
// elements' (x, row) once; for the moving side it also keeps the z-independent part of each
// element's source coordinate, so a plane costs 3 integer adds per sample before the gather.
template <int LC>
constexpr int xrow_stride() { return LC > 0 ? kRowsX + 1 : kRowsX; }
// row stride (floats) of the field stage's NGF rows in LDS: nx rounded up to 4 mod 32
__host__ __device__ constexpr int ng_stride(int nx) { return nx + (36 - nx % 32) % 32; }

// DBG: also copy the product fields to dbg_prod (the field-stage parity check; built only with
// the run-time plan, LC = 0, whose fields are the same).  The hot instances then hold no global
// stores beside their half-spectrum stores: the compiler waits for pending stores before
// reusing their registers, which would stall the transforms.
template <bool MOVING, int LC, bool HALF, bool DBG = false, typename V = float2>
__global__ __launch_bounds__(kThreadsF) void k_fields_x(
    const float* __restrict__ vol, const uint8_t* __restrict__ umask, int nx, int ny, int nz, int tz, int nslots,
    int nf, const int* __restrict__ rotq, float eps, FftPlan pl, const V* __restrict__ twtab,
    V* __restrict__ out, int H, int Hp, long long out_slot_stride,
    uint8_t* __restrict__ mask_out, long long mask_slot_stride, float* __restrict__ dbg_prod) {
  constexpr int T = kThreadsF;
  constexpr int TY = kRowsX;
  constexpr int WS = xrow_stride<LC>();
  constexpr int HR = TY + 2;
  // largest row this instance can see: nx <= Px, and nx <= Px / 2 when HALF; Px = LC when
  // the length is compiled in (the host checks nx against Px before launching)
  constexpr int NXM = LC > 0 ? (HALF ? LC / 2 : LC) : kMaxLen;
  constexpr int PXM = LC > 0 ? LC : kMaxLen;
  // halo-plane samples go to the threads in blocks of kGatherBW columns x HR rows, so a wave
  // gathers a compact patch of the plane (16 x 4 samples) whose rotated source footprint in B
  // spans few cache lines; the LDS plane stays row-major
  constexpr int BW = kGatherBW;
  constexpr int NXP = (NXM + BW - 1) / BW * BW;
  constexpr int ME = (HR * NXP + T - 1) / T;          // halo-plane samples per thread
  constexpr int MN = (TY * NXM + T - 1) / T;          // slice voxels per thread
  constexpr int MU = (TY * (PXM / 2) + T - 1) / T;    // half-spectrum bins per thread
  extern __shared__ __align__(16) unsigned char smem[];
  const int Px = pl.L;
  const int plane = HR * nx;
  const int plane_el = (nx + BW - 1) / BW * BW * HR;   // sample slots, padding columns included
  using S = scalar_t<V>;
  V* tw = reinterpret_cast<V*>(smem);
  V* buf = reinterpret_cast<V*>(smem + align16(sizeof(V) * Px));
  float* val = reinterpret_cast<float*>(smem + align16(sizeof(V) * Px) + align16(sizeof(V) * Px * (TY + 1)));
  float* ng = reinterpret_cast<float*>(reinterpret_cast<unsigned char*>(val) + align16(sizeof(float) * 3 * plane));
  // NGF rows are nxs = nx padded to 4 mod 32 floats apart: the transform's producer reads 8
  // rows x 4 columns per half wave, which then fall into 32 distinct LDS banks
  const int nxs = ng_stride(nx);
  // XCD-aware order (hardware deals block b to XCD b % 8): each XCD walks a contiguous run
  // of (y tile, z chunk, slot) with the y tile fastest, so neighbouring tiles' source
  // footprints in B meet in the same L2.
  const int nyt = (ny + TY - 1) / TY, nzc = (nz + tz - 1) / tz;
  const int nb8 = gridDim.x;
  const int logical = ((int)blockIdx.x % 8) * (nb8 / 8) + (int)blockIdx.x / 8;
  if (logical >= nyt * nzc * nslots) return;
  const int y0 = (logical % nyt) * TY;
  const int z0 = ((logical / nyt) % nzc) * tz;
  const int slot = logical / (nyt * nzc);
  load_twiddles<LC>(tw, twtab, pl);
  const float eps2 = eps * eps;
  const long nv = (long)nx * ny * nz;
  const unsigned tid = threadIdx.x;
  const float qnan = __builtin_nanf("");

  // the volume: on the moving side its copy in bricks, on the fixed side as laid out
  const int nbx = brick_count(nx), nby = brick_count(ny);
  const RView src(vol, MOVING ? 4LL * kBrickVals * nbx * nby * brick_count(nz) : 4LL * nv);

  // ---- per-thread decode of the halo-plane samples
  // moving: source coordinate p 2^17 = k (2 x - (n - 1)) + (n - 1) 2^16 per axis (Q16 matrix k),
  // split into the part fixed by (x, row) and the part of the plane's z; rows outside the
  // grid get a coordinate far below 0, so the box test rejects them.
  // fixed: the voxel's offset within a plane, -1 outside the grid.
  const int* kq = MOVING ? rotq + 9 * slot : nullptr;
  int cx[ME], cy[ME], cz[ME], pe[ME];   // pe: the sample's LDS index in the plane, -1 for none
#pragma unroll
  for (int u = 0; u < ME; ++u) {
    const int e = (int)tid + u * T;
    const int b = e / (BW * HR), w = e - b * (BW * HR);
    const int r = w / BW, x = b * BW + (w - r * BW);
    const int yy = y0 + r - 1;
    const bool slot_ok = e < plane_el && x < nx;
    pe[u] = slot_ok ? r * nx + x : -1;
    const bool in = slot_ok && yy >= 0 && yy < ny;
    if (MOVING) {
      const int dx = 2 * x - (nx - 1), dy = 2 * yy - (ny - 1);
      cx[u] = in ? kq[0] * dx + kq[1] * dy + (nx - 1) * 65536 : -(1 << 30);
      cy[u] = kq[3] * dx + kq[4] * dy + (ny - 1) * 65536;
      cz[u] = kq[6] * dx + kq[7] * dy + (nz - 1) * 65536;
    } else {
      cx[u] = in ? yy * nx + x : -1;
      cy[u] = cz[u] = 0;
    }
  }

  // sample halo plane zz (rows y0-1 .. y0+TY) into ring slot (zz - z0 + 1) mod 3, in groups
  // of HU samples whose gathers are issued before any is used
  auto fill_plane = [&](int zz) {
    float* pv = val + ((zz - z0 + 1) % 3) * plane;
    const bool zin = zz >= 0 && zz < nz;
    const int dz = 2 * zz - (nz - 1);
    const int ax = MOVING ? kq[2] * dz : 0, ay = MOVING ? kq[5] * dz : 0, az = MOVING ? kq[8] * dz : 0;
    const int limx = (nx - 1) << 17, limy = (ny - 1) << 17, limz = (nz - 1) << 17;
    const uint32_t sy4 = 4u * nx, sz4 = 4u * nx * ny;   // byte strides of B along y and z
    constexpr int HU = kGatherGroup;
#pragma unroll
    for (int u0 = 0; u0 < ME; u0 += HU) {
      if (u0 * T >= plane_el) break;
      float v[HU];
      if constexpr (MOVING) {
        float2 c[HU][4];
        float fx[HU], fy[HU], fz[HU];
        bool good[HU];
#pragma unroll
        for (int h = 0; h < HU; ++h) {
          const int u = u0 + h < ME ? u0 + h : ME - 1;
          const int px = cx[u] + ax, py = cy[u] + ay, pz = cz[u] + az;
          const bool ok = zin & ((unsigned)px <= (unsigned)limx) & ((unsigned)py <= (unsigned)limy) &
                          ((unsigned)pz <= (unsigned)limz);
          int ix = px >> 17, iy = py >> 17, iz = pz >> 17;
          const float q = 1.0f / 131072.0f;
          fx[h] = (float)(px & 0x1FFFF) * q;
          fy[h] = (float)(py & 0x1FFFF) * q;
          fz[h] = (float)(pz & 0x1FFFF) * q;
          // p on the upper face: use the last cell with weight 1 on its far corner
          if (ix == nx - 1) { ix = nx - 2; fx[h] = 1.0f; }
          if (iy == ny - 1) { iy = ny - 2; fy[h] = 1.0f; }
          if (iz == nz - 1) { iz = nz - 2; fz[h] = 1.0f; }
          // the cell's brick and its place in it
          const unsigned brick = mad24u(mad24u((unsigned)iz >> 2, nby, (unsigned)iy >> 2), nbx, (unsigned)ix >> 2);
          const unsigned ob = mad24u(brick, kBrickVals,
                                     mad24u(mad24u((unsigned)iz & 3u, 5, (unsigned)iy & 3u), 5, (unsigned)ix & 3u));
          const unsigned o4 = ok ? 4u * ob : kNoOff;
          c[h][0] = src.ld2(o4, 0);          // corners (x, x+1) of the 4 (y, z) edges
          c[h][1] = src.ld2(o4, 4 * 5);
          c[h][2] = src.ld2(o4, 4 * 25);
          c[h][3] = src.ld2(o4, 4 * 30);
          good[h] = ok;
          if (umask) {
            // all 8 corners inside the mask: the smallest of the 8 bytes is nonzero
            const RView srcm(umask, nv);
            const unsigned o = mad24u(mad24u((unsigned)iz, ny, (unsigned)iy), nx, (unsigned)ix);
            const unsigned om = ok ? o : kNoOff;
            unsigned mn = min(srcm.ld1(om, 0), srcm.ld1(om + 1, 0));
            mn = min(mn, min(srcm.ld1(om, sy4 / 4), srcm.ld1(om + 1, sy4 / 4)));
            mn = min(mn, min(srcm.ld1(om, sz4 / 4), srcm.ld1(om + 1, sz4 / 4)));
            mn = min(mn, min(srcm.ld1(om, (sz4 + sy4) / 4), srcm.ld1(om + 1, (sz4 + sy4) / 4)));
            good[h] = ok && mn != 0;
          }
        }
#pragma unroll
        for (int h = 0; h < HU; ++h) {
          const float c00 = lerp_exact(c[h][0].x, c[h][0].y, fx[h]);
          const float c10 = lerp_exact(c[h][1].x, c[h][1].y, fx[h]);
          const float c01 = lerp_exact(c[h][2].x, c[h][2].y, fx[h]);
          const float c11 = lerp_exact(c[h][3].x, c[h][3].y, fx[h]);
          const float c0 = lerp_exact(c00, c10, fy[h]);
          const float c1 = lerp_exact(c01, c11, fy[h]);
          v[h] = good[h] ? lerp_exact(c0, c1, fz[h]) : qnan;
        }
      } else {
#pragma unroll
        for (int h = 0; h < HU; ++h) {
          const int u = u0 + h < ME ? u0 + h : ME - 1;
          const bool ok = zin && cx[u] >= 0;
          const unsigned o = ok ? (unsigned)(zz * ny * nx + cx[u]) : kNoOff / 4;
          const float s = src.ldf(ok ? 4u * o : kNoOff);
          const bool good = ok && (!umask || RView(umask, nv).ld1(o) != 0);
          v[h] = good ? s : qnan;
        }
      }
#pragma unroll
      for (int h = 0; h < HU; ++h) {
        const int u = u0 + h < ME ? u0 + h : ME - 1;
        if (u0 + h < ME && pe[u] >= 0) pv[pe[u]] = v[h];
      }
    }
  };

  // ---- per-thread decode of the slice voxels and of the half-spectrum bins
  int sx[MN], sr[MN];
#pragma unroll
  for (int u = 0; u < MN; ++u) {
    const int e = (int)tid + u * T;
    sx[u] = e % nx;
    sr[u] = e / nx;
  }
  int bk[MU], br[MU];
#pragma unroll
  for (int u = 0; u < MU; ++u) {
    const int e = (int)tid + u * T;
    bk[u] = e % H;
    br[u] = e / H;
  }
  const uint32_t hpb = (uint32_t)sizeof(V) * (uint32_t)Hp;

  // zi = -2, -1 only sample the first two halo planes (z0 - 1, z0)
#pragma unroll 1
  for (int zi = -2; zi < tz; ++zi) {
    const int z = z0 + zi;
    if (z >= nz) break;
    // keep the decoded values opaque per iteration: otherwise the compiler hoists every
    // per-element predicate out of the loop as a 64-bit lane mask and runs out of scalar
    // registers
#pragma unroll
    for (int u = 0; u < ME; ++u) {
      pe[u] = (int)opaque_idx((unsigned)pe[u]);
      cx[u] = (int)opaque_idx((unsigned)cx[u]);
      if (MOVING) {
        cy[u] = (int)opaque_idx((unsigned)cy[u]);
        cz[u] = (int)opaque_idx((unsigned)cz[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < MN; ++u) {
      sx[u] = (int)opaque_idx((unsigned)sx[u]);
      sr[u] = (int)opaque_idx((unsigned)sr[u]);
    }
#pragma unroll
    for (int u = 0; u < MU; ++u) {
      bk[u] = (int)opaque_idx((unsigned)bk[u]);
      br[u] = (int)opaque_idx((unsigned)br[u]);
    }
    fill_plane(z + 1);
    if (zi < 0) continue;
    __syncthreads();
    // mask and NGF of slice z (n = 0 where the eroded mask is 0): the voxel and its six
    // neighbours must be valid samples, i.e. no NaN among the stencil's values
    {
      const float* vm = val + ((zi + 0) % 3) * plane;  // slice z - 1
      const float* vc = val + ((zi + 1) % 3) * plane;  // slice z
      const float* vp = val + ((zi + 2) % 3) * plane;  // slice z + 1
#pragma unroll
      for (int u = 0; u < MN; ++u) {
        const int e = (int)tid + u * T;
        if (u * T >= TY * nx) break;
        if (e < TY * nx) {
          const int x = sx[u], r = sr[u];
          const int c = e + nx;   // (r + 1) * nx + x
          const float gx = 0.5f * (vc[c + 1] - vc[c - 1]);
          const float gy = 0.5f * (vc[c + nx] - vc[c - nx]);
          const float gz = 0.5f * (vp[c] - vm[c]);
          const bool m = x >= 1 && x <= nx - 2 && !__builtin_isnan(vc[c]) && !__builtin_isnan(gx) &&
                         !__builtin_isnan(gy) && !__builtin_isnan(gz);
          float n0 = 0.f, n1 = 0.f, n2 = 0.f;
          if (m) {
            // hardware reciprocal square root (within 1 ulp; its argument is >= eps^2, normal)
            const float inv = __builtin_amdgcn_rsqf(gx * gx + gy * gy + gz * gz + eps2);
            n0 = gx * inv;
            n1 = gy * inv;
            n2 = gz * inv;
          }
          const int q = (int)mad24u((unsigned)r, nxs, (unsigned)x);
          ng[q] = n0;
          ng[TY * nxs + q] = n1;
          ng[2 * TY * nxs + q] = n2;
          if (mask_out) {
            const int yy = y0 + r;
            const unsigned mo = mad24u(mad24u((unsigned)z, ny, (unsigned)yy), nx, (unsigned)x);
            RView(mask_out + slot * mask_slot_stride, nv).st1(yy < ny ? mo : kNoOff, m ? 1 : 0);
          }
        }
      }
    }
    __syncthreads();
    const bool sq = nf != 3;
    if (DBG && dbg_prod && slot == 0) {
      // debug copy of the product fields of slot 0 (same arithmetic as the transform's inputs)
      for (int e = tid; e < TY * nx; e += T) {
        const int r = e / nx, x = e - r * nx, yy = y0 + r;
        if (yy >= ny) continue;
        const int q = r * nxs + x;
        const float n0 = ng[q], n1 = ng[TY * nxs + q], n2 = ng[2 * TY * nxs + q];
        const long vox = ((long)z * ny + yy) * nx + x;
        if (sq) {
          const float f[6] = {n0 * n0, n1 * n1, n2 * n2, n0 * n1, n0 * n2, n1 * n2};
          for (int k = 0; k < 6; ++k) dbg_prod[k * nv + vox] = f[k];
        } else {
          dbg_prod[vox] = n0;
          dbg_prod[nv + vox] = n1;
          dbg_prod[2 * nv + vox] = n2;
        }
      }
    }
    // 6 fields (squared measure): (xx,yy), (zz,xy), (xz,yz); 3 fields (unsquared): (x,y), (z,-).
    // The eroded mask is 0 on the grid's border planes, so the fields vanish there: X1 keeps
    // only the interior slices 1 .. nz-2 and rows 1 .. ny-2, and border slices skip the
    // transform.  (A and B are both shifted by one row and slice, which leaves their
    // correlation unchanged.)
    const int npairs = (z == 0 || z == nz - 1) ? 0 : (nf + 1) / 2;
#pragma unroll 1
    for (int pair = 0; pair < npairs; ++pair) {
      // field selection by workgroup-uniform selects, not branches, so the LDS reads of all
      // of a butterfly's elements are in flight together:
      //   squared:   fa = (p1 ? n2 : n0) (p0 ? n0 : n2),  fb = n1 (p0 ? n1 : p1 ? n0 : n2)
      //   unsquared: fa = (p1 ? n2 : n0),                 fb = n1 (p0 ? 1 : 0)
      const bool p0 = pair == 0, p1 = pair == 1;
      auto products = [&](int x0, int x1, int r) -> V {
        const int x = x0 + x1;
        // x >= nx reads past the row (at most Px floats past ng: the LDS layout pads it) and
        // is replaced by zero below
        const unsigned b = opaque_base(mad24u((unsigned)r, nxs, (unsigned)x0));
        const float n0 = ng[b + x1], n1 = ng[TY * nxs + b + x1], n2 = ng[2 * TY * nxs + b + x1];
        const float a1 = p1 ? n2 : n0;
        const float a2 = sq ? (p0 ? n0 : n2) : 1.0f;
        const float b2 = sq ? (p0 ? n1 : p1 ? n0 : n2) : (p0 ? 1.0f : 0.0f);
        const float fa = a1 * a2, fb = n1 * b2;
        return x < nx ? cplx<V>(fa, fb) : czero<V>();
      };
      auto none = [](int, int, int, V, int) {};
      fft_io<LC, TY, T, false, false, true, WS, HALF>(buf, tw, pl, products, none);
      __syncthreads();
      // split the packed transform: Fa = (Z_k + conj Z_{P-k}) / 2, Fb = -i (Z_k - conj Z_{P-k}) / 2
      // for bins 1 .. Px/2 - 1; bin 0 stores DC + i Nyquist of each field (Fa: Z_0.x + i Z_h.x,
      // Fb: Z_0.y + i Z_h.y with h = Px/2)
      const long long fbase = (long long)(nz - 2) * (ny - 2) * Hp;   // elements per field
      const long long fbytes = (long long)sizeof(V) * fbase;
      const RView oa(out + slot * out_slot_stride + (2 * pair) * fbase, fbytes);
      const RView ob(out + slot * out_slot_stride + (2 * pair + 1) * fbase, 2 * pair + 1 < nf ? fbytes : 0);
      const int row0 = (z - 1) * (ny - 2) + y0 - 1;   // X1 row of grid row y0 (interior rows)
      // predicated rather than branched, so the LDS reads of all of a thread's bins are in
      // flight together: elements past TY * H read row 0 and store nothing
#pragma unroll
      for (int u = 0; u < MU; ++u) {
        if (u * T >= TY * H) break;
        const int e = (int)tid + u * T;
        const bool ok = e < TY * H;
        const int k = ok ? bk[u] : 0, r = ok ? br[u] : 0;
        const V zk = buf[mul24c<WS>((unsigned)k) + r];
        const V zc = buf[mul24c<WS>((unsigned)(k ? Px - k : Px / 2)) + r];
        const int yy = y0 + r;
        const uint32_t off = offv_if<V>(ok && yy >= 1 && yy <= ny - 2, row0 + r, hpb, k);
        oa.template stv<V>(off, k ? cplx<V>(S(0.5) * (zk.x + zc.x), S(0.5) * (zk.y - zc.y)) : cplx<V>(zk.x, zc.x));
        ob.template stv<V>(off, k ? cplx<V>(S(0.5) * (zk.y + zc.y), S(0.5) * (zc.x - zk.x)) : cplx<V>(zk.y, zc.y));
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------------------ y passes
// Pencils along the middle axis.  Workgroup (x-tile, group g, slot): input rows i < n_in of
// in[g], zero beyond; output row c takes transform row (c + out_off) mod L.  HALF: n_in <= L/2
// (first stage pruned).
template <bool INV, int LC, bool HALF, typename V = float2>
__global__ __launch_bounds__(kThreadsP<INV>) void k_pencil(
    const V* __restrict__ in, V* __restrict__ out, int n_in, int n_out, int out_off,
    FftPlan pl, const V* __restrict__ twtab, int H, int Hp, long long in_gstride,
    long long out_gstride, long long in_sstride, long long out_sstride, const uint8_t* __restrict__ flags,
    long long flag_sstride, int ngroups) {
  using S = scalar_t<V>;
  constexpr int W = kTileP<INV>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int L = pl.L;
  // flags (inverse pass only): group g is skipped when flags[g] == 0; output row c of group g
  // is stored only when flags[ngroups + g * n_out + c] != 0.
  const uint8_t* fl = flags ? flags + blockIdx.z * flag_sstride : nullptr;
  if (fl && !fl[blockIdx.y]) return;
  const uint8_t* rowfl = fl ? fl + ngroups + (long long)blockIdx.y * n_out : nullptr;
  V* tw = reinterpret_cast<V*>(smem);
  V* buf = reinterpret_cast<V*>(smem + align16(sizeof(V) * L));
  const int kx0 = blockIdx.x * W;
  // views from this tile's first element to the end of its group (rows n_in resp. n_out)
  const RView src(in + blockIdx.z * in_sstride + blockIdx.y * in_gstride + kx0, (long long)sizeof(V) * ((long long)n_in * Hp - kx0));
  const RView dst(out + blockIdx.z * out_sstride + blockIdx.y * out_gstride + kx0,
                  (long long)sizeof(V) * ((long long)n_out * Hp - kx0));
  const uint32_t rsb = (uint32_t)sizeof(V) * (uint32_t)Hp;
  load_twiddles<LC>(tw, twtab, pl);
  // inverse with flags: the group's row flags go to LDS once (rows c >= n_out read 0), so the
  // last stage's stores need no global load each
  uint8_t* rfl = reinterpret_cast<uint8_t*>(smem + align16(sizeof(V) * L) + align16(sizeof(V) * L * W));
  if (INV && rowfl) {
    const RView rflag(rowfl, n_out);
    for (int c = threadIdx.x; c < L; c += kThreadsP<INV>) rfl[c] = (uint8_t)rflag.ld1((uint32_t)c);
    __syncthreads();
  } else if (LC == 0) {
    __syncthreads();
  }
  // rows i >= n_in lie past the input view and load zero; rows c >= n_out past the output
  // view (and its flag view) and are dropped; columns >= H are masked by kNoOff
  constexpr int T = kThreadsP<INV>;
  auto load = [&](int i0, int i1, int p) -> V {
    const uint32_t b = offv_if<V>(kx0 + p < H, i0, rsb, p);
    return src.template ldv<V, true>(b + (uint32_t)i1 * rsb);
  };
  auto store = [&](int k0, int k1, int p, V v, int) {
    int c = k0 + k1 - out_off;
    if (c < 0) c += L;
    bool keep = kx0 + p < H;
    if constexpr (INV) keep = keep & (!rowfl | (rfl[c] != 0));   // the flag region exists for the inverse
    dst.template stv<V>(offv_if<V>(keep, c, rsb, p), v);
  };
  if (kx0 != 0) {
    fft_io<LC, W, T, INV, false, false, W, HALF>(buf, tw, pl, load, store);
    return;
  }
  // tile 0: its first pencil is the packed DC/Nyquist column
  const int half = L / 2;
  if constexpr (!INV) {
    // forward (out_off = 0, all rows kept): transform into LDS, then split the packed pencil,
    // Y = D + i N: row c < L/2 takes D(c) = (Y(c) + conj Y(-c)) / 2, row L - c takes
    // N(c) = -i (Y(c) - conj Y(-c)) / 2; rows 0 and L/2 keep Y
    fft_io<LC, W, T, false, false, true, W, HALF>(buf, tw, pl, load, [](int, int, int, V, int) {});
    __syncthreads();
    for (int e = threadIdx.x; e < L * W; e += T) {
      const int c = e / W, p = e - c * W;
      V v = buf[e];
      if (p == 0 && c != 0 && c != half) {
        const V m = buf[(L - c) * W];
        v = c < half ? cplx<V>(S(0.5) * (v.x + m.x), S(0.5) * (v.y - m.y))
                     : cplx<V>(S(0.5) * (v.y + m.y), S(0.5) * (v.x - m.x));
      }
      dst.template stv<V>(offv_if<V>(kx0 + p < H, c, rsb, p), v);
    }
  } else {
    // inverse: the input rows are S_D(ky) for ky < L/2 and S_N(L - ky) above (rows 0 and
    // L/2: S_D + i S_N); transform G(ky) = S_D(ky) + i S_N(ky), using the Hermitian symmetry
    // of both planes for the rows that are not stored
    fft_io<LC, W, T, true, false, false, W, false>(
        buf, tw, pl,
        [&](int i0, int i1, int p) -> V {
          // branch-free, so a butterfly's loads are all in flight together
          const V s = load(i0, i1, p);
          const int i = i0 + i1;
          const bool mix = p == 0 && i != 0 && i != half;
          const V m = src.template ldv<V, false>(offv_if<V>(mix, L - i, rsb, 0));
          const V g = i < half ? cplx<V>(s.x - m.y, s.y + m.x) : cplx<V>(m.x + s.y, s.x - m.y);
          return mix ? g : s;
        },
        store);
  }
}

// ------------------------------------------------------------------------------ z pass
// Workgroup (ky, x-tile, slot), ordered so that the slots of one tile run back to back on
// one XCD and share that tile of A's spectra through its L2.  Per field: z forward with
// the multiply-accumulate against A's conjugate spectrum done on the last stage's
// registers; then the sum goes through LDS once for the z inverse, whose last stage
// stores the kept displacement rows.
// PACKED: a separate launch of 2 workgroups per slot for tile 0 at ky = 0 and Py/2, whose
// first pencil is the packed DC/Nyquist column (see the top of this file); the main launch
// skips those two tiles.  Kept apart so the main kernel's register budget is unchanged.
template <int LC, bool HALF, bool PACKED, typename V = float2>
__global__ __launch_bounds__(kThreadsZ) void k_zpass(
    const V* __restrict__ X2, const V* __restrict__ spec, V* __restrict__ Y3,
    int nz, int Py, int H, int Hp, int Wz, int out_off, FftPlan pl, const V* __restrict__ twtab,
    long long x2_sstride, long long y3_sstride, int ntiles, int nslots, int nreal,
    const uint8_t* __restrict__ flags, long long flag_sstride, int nf) {
  using S = scalar_t<V>;
  constexpr int W = kTileW;
  constexpr int NSLOT = consumer_slots<LC, W, kThreadsZ>();
  extern __shared__ __align__(16) unsigned char smem[];
  const int Pz = pl.L;
  V* tw = reinterpret_cast<V*>(smem);
  V* buf = reinterpret_cast<V*>(smem + align16(sizeof(V) * Pz));
  int slot, ky, kx0;
  if constexpr (PACKED) {
    if ((int)blockIdx.x >= 2 * nslots) return;
    slot = blockIdx.x % nslots;
    ky = blockIdx.x < nslots ? 0 : Py / 2;
    kx0 = 0;
  } else {
    // XCD-aware order: hardware deals block b to XCD b % 8; give each XCD a contiguous run.
    const int nb8 = gridDim.x;
    const int b = blockIdx.x;
    const int logical = (b % 8) * (nb8 / 8) + b / 8;
    if (logical >= nreal) return;
    slot = logical % nslots;
    const int rest = logical / nslots;
    const int tile = rest % ntiles;
    ky = rest / ntiles;
    kx0 = tile * W;
    if (kx0 == 0 && (ky == 0 || 2 * ky == Py)) return;   // done by the PACKED launch
  }
  load_twiddles<LC>(tw, twtab, pl);
  if (LC == 0) __syncthreads();
  const long long fstride_x2 = (long long)nz * Py * Hp;
  const long long fstride_sp = (long long)Pz * Py * Hp;
  const long long zs = (long long)Py * Hp;
  const long long col0 = (long long)ky * Hp + kx0;
  const uint32_t zsb = (uint32_t)sizeof(V) * (uint32_t)zs;
  // views from this pencil tile to the end of field f: moving input (rows i >= nz lie past
  // it and load zero) and A's spectrum; masked columns load zero and are never stored
  auto src_view = [&](int f) { return RView(X2 + slot * x2_sstride + f * fstride_x2 + col0, (long long)sizeof(V) * (fstride_x2 - col0)); };
  auto spec_view = [&](int f) { return RView(spec + f * fstride_sp + col0, (long long)sizeof(V) * (fstride_sp - col0)); };
  auto loader = [&](const RView& src) {
    return [&src, kx0, H, zsb](int i0, int i1, int p) -> V {
      const uint32_t b = offv_if<V>(kx0 + p < H, i0, zsb, p);
      return src.template ldv<V, true>(b + (uint32_t)i1 * zsb);
    };
  };
  if constexpr (!PACKED) {
    V acc[NSLOT];
#pragma unroll
    for (int u = 0; u < NSLOT; ++u) acc[u] = czero<V>();
#pragma unroll 1
    for (int f = 0; f < nf; ++f) {
      const RView src = src_view(f);
      const RView a = spec_view(f);
      fft_io<LC, W, kThreadsZ, false, false, false, W, HALF>(
          buf, tw, pl, loader(src),
          [&](int k0, int k1, int p, V v, int sl) {
            const uint32_t b = offv_if<V>(kx0 + p < H, k0, zsb, p);
            const V sv = a.template ldv<V, false>(b + (uint32_t)k1 * zsb);
            acc[sl].x = fmadd(v.x, sv.x, fmadd(-v.y, sv.y, acc[sl].x));
            acc[sl].y = fmadd(v.x, sv.y, fmadd(v.y, sv.x, acc[sl].y));
          });
      __syncthreads();
    }
    if constexpr (LC > 0) {
      for_each_last_slot<LC, W, kThreadsZ>([&](int k, int p, int sl) { buf[k * W + p] = acc[sl]; });
    } else {
      int sl = 0;
      for (int e = threadIdx.x; e < Pz * W; e += kThreadsZ, ++sl) buf[e] = acc[sl];
    }
  } else {
    // tile 0 at ky = 0 or Py/2: its first pencil holds D + i N with D, N real along z, so its
    // z transform is Z = D^ + i N^ with both parts Hermitian in kz.  Split Z with Z(-kz), take
    // A's D and N spectra from the same split stored by k_zstore, and accumulate
    // conj(A_D) B_D + i conj(A_N) B_N, whose z inverse is (D-plane sum) + i (Nyquist-plane sum).
    constexpr int NE = ((LC > 0 ? LC : kMaxLen) * W + kThreadsZ - 1) / kThreadsZ;
    V acc[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) acc[u] = czero<V>();
    const int hz = Pz / 2;
#pragma unroll 1
    for (int f = 0; f < nf; ++f) {
      const RView src = src_view(f);
      const RView a = spec_view(f);
      fft_io<LC, W, kThreadsZ, false, false, true, W, HALF>(buf, tw, pl, loader(src),
                                                          [](int, int, int, V, int) {});
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int e = (int)threadIdx.x + u * kThreadsZ;
        if (e < Pz * W) {
          const int kz = e / W, p = e - kz * W;
          const V v = buf[e];
          const V sk = a.template ldv<V, false>(offv_if<V>(kx0 + p < H, kz, zsb, p));
          if (p != 0) {
            acc[u].x = fmadd(v.x, sk.x, fmadd(-v.y, sk.y, acc[u].x));
            acc[u].y = fmadd(v.x, sk.y, fmadd(v.y, sk.x, acc[u].y));
          } else {
            const int m = kz ? Pz - kz : 0;
            const V vm = buf[m * W];
            const V sm = a.template ldv<V, false>(offv<V>(m, zsb, 0));
            const V bd = cplx<V>(S(0.5) * (v.x + vm.x), S(0.5) * (v.y - vm.y));   // B_D(kz)
            const V bn = cplx<V>(S(0.5) * (v.y + vm.y), S(0.5) * (vm.x - v.x));   // B_N(kz)
            V ad, an;   // w conj(A_D(kz)), w conj(A_N(kz))
            if (kz == 0 || kz == hz) {
              ad = cplx<V>(sk.x, S(0));
              an = cplx<V>(-sk.y, S(0));
            } else if (kz < hz) {
              ad = sk;
              an = sm;
            } else {
              ad = cplx<V>(sm.x, -sm.y);
              an = cplx<V>(sk.x, -sk.y);
            }
            const V t1 = cplx<V>(ad.x * bd.x - ad.y * bd.y, ad.x * bd.y + ad.y * bd.x);
            const V t2 = cplx<V>(an.x * bn.x - an.y * bn.y, an.x * bn.y + an.y * bn.x);
            acc[u].x += t1.x - t2.y;
            acc[u].y += t1.y + t2.x;
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = (int)threadIdx.x + u * kThreadsZ;
      if (e < Pz * W) buf[e] = acc[u];
    }
  }
  __syncthreads();
  const RView dst(Y3 + slot * y3_sstride + col0, (long long)sizeof(V) * ((long long)Wz * zs - col0));
  // kept-row flags to LDS (rows c >= Wz read 0); the inverse's stage barriers order these
  // writes before the last stage reads them
  uint8_t* zfl = reinterpret_cast<uint8_t*>(smem + align16(sizeof(V) * Pz) + align16(sizeof(V) * Pz * W));
  {
    const RView zflag(flags + slot * flag_sstride, Wz);
    for (int c = threadIdx.x; c < Pz; c += kThreadsZ) zfl[c] = (uint8_t)zflag.ld1((uint32_t)c);
    __syncthreads();
  }
  fft_io<LC, W, kThreadsZ, true, true, false>(
      buf, tw, pl, [](int, int, int) { return czero<V>(); },
      [&](int k0, int k1, int p, V v, int) {
        int c = k0 + k1 - out_off;
        if (c < 0) c += Pz;
        const bool keep = (kx0 + p < H) & (zfl[c] != 0);   // no short-circuit: no branch per element
        dst.template stv<V>(offv_if<V>(keep, c, zsb, p), v);
      });
}

// Fixed side: z forward of A's fields, stored as w_f * scale * conj(.) in spec[f][kz][ky][kx]
// (w_f = 2 for the cross products of the squared measure, else 1).
template <int LC, typename V = float2>
__global__ __launch_bounds__(kThreads) void k_zstore(
    const V* __restrict__ X2, V* __restrict__ spec, int nz, int Py, int H, int Hp,
    FftPlan pl, const V* __restrict__ twtab, scalar_t<V> scale, int nf) {
  using S = scalar_t<V>;
  constexpr int W = kTileW;
  extern __shared__ __align__(16) unsigned char smem[];
  const int Pz = pl.L;
  V* tw = reinterpret_cast<V*>(smem);
  V* buf = reinterpret_cast<V*>(smem + align16(sizeof(V) * Pz));
  const int kx0 = blockIdx.x * W;
  const int ky = blockIdx.y;
  const int f = blockIdx.z;
  load_twiddles<LC>(tw, twtab, pl);
  if (LC == 0) __syncthreads();
  const long long zs = (long long)Py * Hp;
  const V* src = X2 + (long long)f * nz * zs + (long long)ky * Hp + kx0;
  const S w = (nf == 6 && f >= 3 ? S(2) : S(1)) * scale;  // Eq. (6) cross terms x2
  V* dst = spec + (long long)f * Pz * zs + (long long)ky * Hp + kx0;
  auto load = [&](int i0, int i1, int p) -> V {
    const int i = i0 + i1;
    return (i < nz && kx0 + p < H) ? src[(long long)i * zs + p] : czero<V>();
  };
  if (kx0 != 0 || (ky != 0 && 2 * ky != Py)) {
    fft_io<LC, W, kThreads, false, false, false>(buf, tw, pl, load, [&](int k0, int k1, int p, V v, int) {
      if (kx0 + p < H) dst[(long long)(k0 + k1) * zs + p] = cplx<V>(w * v.x, -w * v.y);
    });
    return;
  }
  // tile 0 at ky = 0 or Py/2: the first pencil transforms to Z = D^ + i N^ (both Hermitian in
  // kz); store D^(kz) at kz in (0, Pz/2), N^(Pz - kz) at kz in (Pz/2, Pz), and Z at 0 and Pz/2
  fft_io<LC, W, kThreads, false, false, true>(buf, tw, pl, load, [](int, int, int, V, int) {});
  __syncthreads();
  const int hz = Pz / 2;
  for (int e = threadIdx.x; e < Pz * W; e += kThreads) {
    const int kz = e / W, p = e - kz * W;
    V v = buf[e];
    if (p == 0 && kz != 0 && kz != hz) {
      const V m = buf[(Pz - kz) * W];
      v = kz < hz ? cplx<V>(S(0.5) * (v.x + m.x), S(0.5) * (v.y - m.y))
                  : cplx<V>(S(0.5) * (v.y + m.y), S(0.5) * (v.x - m.x));
    }
    if (kx0 + p < H) dst[(long long)kz * zs + p] = cplx<V>(w * v.x, -w * v.y);
  }
}

// ------------------------------------------------------------------------------ moving mask runs
// Without a user mask on B the eroded mask of B^ depends only on the rotation, and on each grid
// row (y, z) it is one run of x.  A sample at grid point (x, y, z) is valid when its Q16 source
// coordinate p_i 2^17 = sum_j k_ij (2 x_j - (n_j - 1)) + (n_i - 1) 2^16 lies in [0, (n_i - 1) 2^17]
// on every axis i: the field stage's integer test.  Along a row p_i = a_i x + b_i (a_i = 2 k_i0),
// so the valid samples form the run [lo, hi] that the three pairs of inequalities leave, found
// with exact integer floor and ceiling divisions (no overflow: |a_i x + b_i| < 2^30).  A grid
// point is in the eroded mask when it is interior and the samples at it and at its six
// neighbours are valid (Sec. 3.1 masks; the central-difference stencil): the run of row (y, z)
// shrunk by one at each end, intersected with the runs of rows (y +- 1, z) and (y, z +- 1).  For
// finite B this is bit for bit the set of voxels whose fields the field stage keeps, so the
// overlap table can be built from the rotations alone, beside the field stage.
__device__ __forceinline__ int floor_div(int a, int b) {   // b > 0
  const int q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}

// the run of valid samples on row (y, z) of B's grid, empty (lo > hi) off the grid.  32-bit
// arithmetic suffices: |k| <= 2^17 (|R_ij| <= 2) and n <= 512 keep |b|, L - b below 2^30.
__device__ __forceinline__ int2 sample_run(const int* __restrict__ kq, int nx, int ny, int nz, int y, int z) {
  if ((unsigned)y >= (unsigned)ny || (unsigned)z >= (unsigned)nz) return make_int2(1, 0);
  const int n[3] = {nx, ny, nz};
  const int dy = 2 * y - (ny - 1), dz = 2 * z - (nz - 1);
  int lo = 0, hi = nx - 1;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int a = 2 * kq[3 * i];
    const int b = -kq[3 * i] * (nx - 1) + kq[3 * i + 1] * dy + (n[i] - 1) * 65536 + kq[3 * i + 2] * dz;
    const int L = (n[i] - 1) << 17;
    if (a == 0) {
      if (b < 0 || b > L) return make_int2(1, 0);
    } else if (a > 0) {   // -b <= a x <= L - b
      lo = max(lo, -floor_div(b, a));
      hi = min(hi, floor_div(L - b, a));
    } else {              // b - L <= |a| x <= b
      lo = max(lo, -floor_div(L - b, -a));
      hi = min(hi, floor_div(b, -a));
    }
  }
  return lo <= hi ? make_int2(lo, hi) : make_int2(1, 0);
}

// runs[slot][z][y] = eroded-mask run of row (y, z) (empty: x > y); grid (ceil(ny nz / kThreads), slots)
__global__ __launch_bounds__(kThreads) void k_mask_runs(const int* __restrict__ rotq, int nx, int ny, int nz,
                                                        int2* __restrict__ runs, long long runs_sstride) {
  const int slot = blockIdx.y;
  const int t = (int)(blockIdx.x * kThreads + threadIdx.x);
  if (t >= ny * nz) return;
  const int z = t / ny, y = t - z * ny;
  const int* kq = rotq + 9 * slot;
  int lo = 1, hi = 0;
  if (y >= 1 && y <= ny - 2 && z >= 1 && z <= nz - 2) {
    const int2 c = sample_run(kq, nx, ny, nz, y, z);
    lo = max(1, c.x + 1);
    hi = min(nx - 2, c.y - 1);
    const int2 r[4] = {sample_run(kq, nx, ny, nz, y - 1, z), sample_run(kq, nx, ny, nz, y + 1, z),
                       sample_run(kq, nx, ny, nz, y, z - 1), sample_run(kq, nx, ny, nz, y, z + 1)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lo = max(lo, r[k].x);
      hi = min(hi, r[k].y);
    }
  }
  runs[slot * runs_sstride + t] = make_int2(lo, hi);
}

// Step 1 of the overlap table from the runs: plane[slot][z][y][x] = sum over rows y' <= y of the
// run's points with x' <= x.  One wave per 64 columns of a slice, walking down its rows.
template <typename PT>
__global__ __launch_bounds__(64) void k_sat_planes_runs(const int2* __restrict__ runs, PT* __restrict__ plane,
                                                        int nx, int ny, long long runs_sstride,
                                                        long long plane_sstride) {
  const int z = blockIdx.y, slot = blockIdx.z;
  const int x = (int)(blockIdx.x * 64 + threadIdx.x);
  if (x >= nx) return;
  const int2* r = runs + slot * runs_sstride + (long long)z * ny;
  PT* out = plane + slot * plane_sstride + (long long)z * ny * nx + x;
  uint32_t col = 0;
#pragma unroll 8
  for (int y = 0; y < ny; ++y) {
    const int2 v = r[y];
    col += (uint32_t)max(0, min(x - v.x + 1, v.y - v.x + 1));   // 0 for an empty run
    out[(long long)y * nx] = (PT)col;
  }
}

// ------------------------------------------------------------------------------ overlap SAT
// sat[slot][(nz+1)][(ny+1)][(nx+1)], zero on index 0 of every axis:
// sat[z+1][y+1][x+1] = sum of mask over [0..z] x [0..y] x [0..x].
// Step 1 (one workgroup per z slice): the slice's 2-D inclusive prefix over (y, x),
// plane[slot][z][y][x] (PT = uint16_t when nx * ny < 65536, which halves the pass's bytes).
// Rows go to the waves (a wave scan per row), then each thread walks its column down a
// group of rows.
constexpr int kSatThreads = 512;
template <typename PT>
__global__ __launch_bounds__(kSatThreads) void k_sat_planes(const uint8_t* __restrict__ mask,
                                                            PT* __restrict__ plane, int nx, int ny,
                                                            long long mask_sstride, long long plane_sstride) {
  constexpr int NW = kSatThreads / 64;  // rows per group
  __shared__ uint32_t rows[NW][kMaxLen];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int z = blockIdx.x, slot = blockIdx.y;
  const long long off = (long long)z * ny * nx;
  const RView m(mask + slot * mask_sstride + off, (long long)ny * nx);
  PT* out = plane + slot * plane_sstride + off;
  uint32_t col = 0;  // running column sum of thread x = threadIdx.x (nx <= kMaxLen = kSatThreads)
  for (int y0 = 0; y0 < ny; y0 += NW) {
    const int y = y0 + wave;
    if (y < ny) {
      // the row's 64-column chunks are all loaded before the first is scanned
      constexpr int NC = kMaxLen / 64;
      uint32_t v[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int x = c * 64 + lane;
        v[c] = m.ld1(x < nx ? (unsigned)(y * nx + x) : kNoOff);  // 0 past the row (no access)
      }
      uint32_t carry = 0;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (c * 64 >= nx) break;
        const int x = c * 64 + lane;
        uint32_t u = v[c];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const uint32_t t = __shfl_up(u, d, 64);
          if (lane >= d) u += t;
        }
        if (x < nx) rows[wave][x] = carry + u;
        carry += __shfl(u, 63, 64);
      }
    }
    __syncthreads();
    const int x = threadIdx.x;
    if (x < nx) {
      for (int r = 0; r < NW && y0 + r < ny; ++r) {
        col += rows[r][x];
        out[(long long)(y0 + r) * nx + x] = (PT)col;
      }
    }
    __syncthreads();
  }
}

// Step 2: prefix over z for every (y, x), written with the zero borders.  Each column is read
// SU planes at a time, all loads issued before the running sum stores them.
template <typename PT>
__global__ __launch_bounds__(kThreads) void k_sat_z(const PT* __restrict__ plane, int* __restrict__ sat,
                                                    int nx, int ny, int nz, long long plane_sstride,
                                                    long long sat_sstride) {
  constexpr int SU = 16;
  const int slot = blockIdx.y;
  const int X = nx + 1, Y = ny + 1;
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= X * Y) return;
  const int yy = t / X, xx = t % X;
  int* s = sat + slot * sat_sstride + t;
  const long long zstep = (long long)Y * X;
  s[0] = 0;
  if (yy == 0 || xx == 0) {
    for (int z = 1; z <= nz; ++z) s[z * zstep] = 0;
    return;
  }
  const PT* p = plane + slot * plane_sstride + (long long)(yy - 1) * nx + (xx - 1);
  const long long pstep = (long long)ny * nx;
  int run = 0;
  for (int z0 = 0; z0 < nz; z0 += SU) {
    uint32_t v[SU];
#pragma unroll
    for (int u = 0; u < SU; ++u) v[u] = z0 + u < nz ? (uint32_t)p[(z0 + u) * pstep] : 0u;
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      run += (int)v[u];
      if (z0 + u < nz) s[(z0 + u + 1) * zstep] = run;
    }
  }
}

struct OverlapGeom {
  int nA[3];   // x, y, z
  int nB[3];
  int lo[3];   // bounding box of A's eroded mask per axis: [1, nA - 2] without a user mask
  int hi[3];   // (lo > hi when the mask is empty)
};

// Count of the moving mask over A's bounding box shifted by chi and clipped to B's grid: the
// exact N(chi) when A's eroded mask is that box (no user mask: [1, nA-2]), else an upper bound.
__device__ __forceinline__ long long box_count(const int* __restrict__ s, const OverlapGeom& g,
                                               int cx, int cy, int cz) {
  const int X = g.nB[0] + 1, Y = g.nB[1] + 1;
  const int lx = max(g.lo[0] + cx, 0), hx = min(g.hi[0] + cx, g.nB[0] - 1);
  const int ly = max(g.lo[1] + cy, 0), hy = min(g.hi[1] + cy, g.nB[1] - 1);
  const int lz = max(g.lo[2] + cz, 0), hz = min(g.hi[2] + cz, g.nB[2] - 1);
  if (lx > hx || ly > hy || lz > hz) return 0;
  auto at = [&](int z, int y, int x) { return (long long)s[((long long)z * Y + y) * X + x]; };
  return at(hz + 1, hy + 1, hx + 1) - at(lz, hy + 1, hx + 1) - at(hz + 1, ly, hx + 1) -
         at(hz + 1, hy + 1, lx) + at(lz, ly, hx + 1) + at(lz, hy + 1, lx) + at(hz + 1, ly, lx) -
         at(lz, ly, lx);
}

__device__ __forceinline__ unsigned int ordered_bits(float f) {
  const unsigned int u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Smallest N that meets the minimum overlap: N >= gamma * m (the product rounded to double,
// N an integer, so N >= ceil(gamma * m)) and N >= 1.
__device__ __forceinline__ long long threshold(long long count_a, long long count_b, double gamma) {
  const long long m = count_a < count_b ? count_a : count_b;
  const double t = ceil(gamma * (double)m);
  const long long tt = (long long)t;
  return tt > 1 ? tt : 1;
}

// ------------------------------------------------------------------------------ gamma pruning
// One (zc, yc) row of k_bounds: its row flag, and for yc = 0 its z-row flag.
__device__ __forceinline__ void bounds_row(const int* __restrict__ sat, const OverlapGeom& g, int Wy, int Wz,
                                           long long sat_sstride, long long count_a, double gamma,
                                           uint8_t* __restrict__ flags, long long flag_sstride, int slot, int t,
                                           bool* rowflag, bool* zflag) {
  const int zc = t / Wy, yc = t % Wy;
  const int* s = sat + slot * sat_sstride;
  const int X = g.nB[0] + 1, Y = g.nB[1] + 1;
  const long long count_b = s[(long long)(g.nB[2] + 1) * Y * X - 1];
  const long long thr = threshold(count_a, count_b, gamma);
  const int cz = zc - (g.nA[2] - 1), cy = yc - (g.nA[1] - 1);
  const int lz = max(g.lo[2] + cz, 0), hz = min(g.hi[2] + cz, g.nB[2] - 1);
  const int ly = max(g.lo[1] + cy, 0), hy = min(g.hi[1] + cy, g.nB[1] - 1);
  uint8_t* f = flags + slot * flag_sstride;
  auto at = [&](int z, int y) { return (long long)s[((long long)z * Y + y) * X + (X - 1)]; };
  long long rb = 0;
  if (lz <= hz && ly <= hy) rb = at(hz + 1, hy + 1) - at(lz, hy + 1) - at(hz + 1, ly) + at(lz, ly);
  *rowflag = rb >= thr;
  f[Wz + t] = *rowflag ? 1 : 0;
  if (yc == 0) {
    long long pb = 0;
    if (lz <= hz) pb = at(hz + 1, Y - 1) - at(lz, Y - 1);
    *zflag = pb >= thr;
    f[zc] = *zflag ? 1 : 0;
  }
}

// Upper bounds of N(chi) from the SAT: over a z-row (all y and x of B) and over a (z, y) row
// (all x of B).  flags[slot] = zflag[Wz] then rowflag[Wz][Wy]; a 0 flag means no displacement
// of that z-row (resp. row) can reach the overlap threshold, so the inverse passes skip it.
// rowstat (optional, measurement): rowstat[0] += flagged z-rows, rowstat[1] += flagged rows.
__global__ __launch_bounds__(kThreads) void k_bounds(const int* __restrict__ sat, OverlapGeom g, int Wy, int Wz,
                                                     long long sat_sstride, long long count_a, double gamma,
                                                     uint8_t* __restrict__ flags, long long flag_sstride,
                                                     unsigned long long* __restrict__ keys,
                                                     unsigned* __restrict__ nwork,
                                                     unsigned long long* __restrict__ rowstat) {
  const int slot = blockIdx.y;
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t == 0) keys[slot] = 0ull;   // the slot's argmax key, maximised by the final pass
  if (t == 0 && slot == 0 && nwork) *nwork = 0u;   // the final pass's work list, built next
  bool rowflag = false, zflag = false;
  if (t < Wz * Wy) bounds_row(sat, g, Wy, Wz, sat_sstride, count_a, gamma, flags, flag_sstride, slot, t,
                              &rowflag, &zflag);
  if (rowstat) {
    // one atomic per wave and counter; every lane of the wave reaches the ballots
    const unsigned long long br = __ballot(rowflag), bz = __ballot(zflag);
    if ((threadIdx.x & 63) == 0) {
      if (br) atomicAdd(rowstat + 1, (unsigned long long)__popcll(br));
      if (bz) atomicAdd(rowstat, (unsigned long long)__popcll(bz));
    }
  }
}


// ------------------------------------------------------------------------------ final x pass
// Workgroup (row group, zc, slot): 8 packed complex pencils = 16 output rows (yc).
// Two real rows with half spectra S1, S2 are recovered at once from Z = S1 + i S2 extended
// by Hermitian symmetry: z = IFFT(Z), S1 row = Re z, S2 row = Im z.  The first FFT stage
// builds Z straight from the two rows; the last stage normalises and reduces in registers.
// Overlaps: for a fixed-side box, N(chi) = D(hx + 1) - D(lx) where D(x) is the 4-corner
// combination of the SAT over the row's z and y ranges; D rows are built in LDS first.
// NCOUNT: the fixed side has a general mask, so N(chi) is read from the exact count rows that
// k_overlap_x wrote (ncount[slot][zc][yc][cx]) instead of the SAT box sums.
template <bool WRITE_MAP, int LC, bool NCOUNT = false, typename V = float2>
__global__ __launch_bounds__(kThreadsC) void k_final_x(
    const V* __restrict__ Y4, const int* __restrict__ sat, unsigned long long* __restrict__ keys,
    OverlapGeom g, int Wx, int Wy, int Wz, int H, int Hp, FftPlan pl, const V* __restrict__ twtab,
    long long y4_sstride, long long sat_sstride, long long count_a, double gamma,
    float* __restrict__ cmap, long long* __restrict__ nmap, const uint8_t* __restrict__ flags,
    long long flag_sstride, const unsigned* __restrict__ work, const unsigned* __restrict__ nwork,
    const int* __restrict__ ncount, long long ncount_sstride) {
  constexpr int T = kThreadsC;
  constexpr int WP = kRowsC;  // packed pencils
  constexpr int NR = 2 * WP;  // output rows
  static_assert(NR <= 32, "row flags are kept as a 32-bit mask");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ unsigned long long red[T / 64];
  const int Px = pl.L;
  const int X1 = g.nB[0] + 1;
  using S = scalar_t<V>;
  V* tw = reinterpret_cast<V*>(smem);
  V* buf = reinterpret_cast<V*>(smem + align16(sizeof(V) * Px));
  int* drow = reinterpret_cast<int*>(smem + align16(sizeof(V) * Px) + align16(sizeof(V) * Px * (WP + 1)));
  // one group of NR displacement rows (slot, zc, yc0 .. yc0 + NR - 1)
  auto run = [&](const int slot, const int zc, const int yc0) {
  const int* s = sat + slot * sat_sstride;
  // rows whose overlap bound is below the threshold hold no valid displacement and were
  // not produced by the inverse passes; without a map to write, skip groups of such rows
  const uint8_t* rowfl = flags + slot * flag_sstride + Wz + (long long)zc * Wy;
  // the NR row flags as one bit mask (bit rr: row yc0 + rr was produced); rows past Wy lie
  // past the flag view and read 0.  All loads are issued before any is used.
  unsigned fmask = 0;
  {
    const RView rf(rowfl, Wy);
    unsigned fl[NR];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) fl[rr] = rf.ld1((uint32_t)(yc0 + rr));
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) fmask |= fl[rr] ? 1u << rr : 0u;
  }
  if (!WRITE_MAP && !fmask) return;
  const int half = Px / 2;
  // D rows: for row rr (yc = yc0 + rr), D(x) = sum of the SAT over the row's z and y ranges
  // up to column x (x = 0 .. nB_x); empty ranges give D = 0.  Rows go to groups of DG
  // threads, columns to the threads of a group.
  if constexpr (!NCOUNT) {
    constexpr int DG = T < 256 ? T : 256;
    constexpr int RG = T / DG;                  // row groups
    constexpr int RPT = (NR + RG - 1) / RG;     // rows per thread
    const int X = X1, Y = g.nB[1] + 1;
    const int cz = zc - (g.nA[2] - 1);
    const int lz = max(g.lo[2] + cz, 0), hz = min(g.hi[2] + cz, g.nB[2] - 1);
    const RView sv(s, 4LL * (g.nB[2] + 1) * Y * X);
    const int rg = (int)threadIdx.x / DG;
    // byte offsets of the 4 SAT rows of each of this thread's rows (the SAT of one slot is
    // far below 2 GiB); kNoOff where the row needs no counts
    uint32_t o[RPT][4];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int rr = rg + i * RG;
      const int cy = yc0 + rr - (g.nA[1] - 1);
      const int ly = max(g.lo[1] + cy, 0), hy = min(g.hi[1] + cy, g.nB[1] - 1);
      // without a map, rows that hold no valid displacement (flag 0) need no counts
      const bool any = rr < NR && lz <= hz && ly <= hy && yc0 + rr < Wy && (WRITE_MAP || ((fmask >> rr) & 1u));
      o[i][0] = any ? 4u * (uint32_t)(((hz + 1) * Y + hy + 1) * X) : kNoOff;
      o[i][1] = any ? 4u * (uint32_t)((lz * Y + hy + 1) * X) : kNoOff;
      o[i][2] = any ? 4u * (uint32_t)(((hz + 1) * Y + ly) * X) : kNoOff;
      o[i][3] = any ? 4u * (uint32_t)((lz * Y + ly) * X) : kNoOff;
    }
    for (int x = (int)threadIdx.x % DG; x < X1; x += DG) {
      const uint32_t x4 = 4u * x;
      int v[RPT][4];
#pragma unroll
      for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[i][q] = sv.ldi(o[i][q] + x4);
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int rr = rg + i * RG;
        if (rr < NR) drow[rr * X1 + x] = v[i][0] - v[i][1] - v[i][2] + v[i][3];
      }
    }
  }
  const long long count_b = s[(long long)(g.nB[2] + 1) * (g.nB[1] + 1) * (g.nB[0] + 1) - 1];
  // counts and canonical indices fit 32 bits: N <= |M_B| < 2^31, W_x W_y W_z < 2^31
  const int thr = (int)threshold(count_a, count_b, gamma);
  const int* nrows = NCOUNT ? ncount + slot * ncount_sstride + ((long long)zc * Wy) * Wx : nullptr;
  if (LC == 0) __syncthreads();
  unsigned long long best = 0ull;
  const RView rows(Y4 + slot * y4_sstride + ((long long)zc * Wy) * Hp, (long long)sizeof(V) * Wy * Hp);  // rows >= Wy load zero
  const uint32_t hpb = (uint32_t)sizeof(V) * (uint32_t)Hp;
  auto pack = [&](int k0, int k1, int p) -> V {
    const int k = k0 + k1;
    const int r0 = yc0 + 2 * p;
    // bin 0 holds DC + i Nyquist of each row.  Branch-free, so the loads of a butterfly's
    // elements are all in flight together.
    const bool lo = k < half;
    const int kk = k == half ? 0 : lo ? k : Px - k;
    const uint32_t o0 = offv<V>(r0, hpb, kk);
    // (cached loads: each bin is read twice, for k and Px - k)
    const V a = rows.template ldv<V, false>((fmask >> (2 * p)) & 1u ? o0 : kNoOff);
    const V c = rows.template ldv<V, false>((fmask >> (2 * p + 1)) & 1u ? o0 + hpb : kNoOff);
    // k < half: S1 + i S2; k > half: conj(S1) + i conj(S2); k = 0 / half: DC / Nyquist
    const S sg = lo ? S(1) : S(-1);
    V z = cplx<V>(fmadd(-sg, c.y, a.x), fmadd(sg, a.y, c.x));
    z = k == 0 ? cplx<V>(a.x, c.x) : z;
    z = k == half ? cplx<V>(a.y, c.y) : z;
    return z;
  };
  auto emit = [&](int j0, int j1, int p, V zv, int) {
    int cx = j0 + j1 + g.nA[0] - 1;   // < 2 Px
    if (cx >= Px) cx -= Px;
    if (cx >= Wx) return;
    const int chx = cx - (g.nA[0] - 1);
    const int lx = max(g.lo[0] + chx, 0), hx = min(g.hi[0] + chx, g.nB[0] - 1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int rr = 2 * p + h;
      const int yc = yc0 + rr;
      if (yc >= Wy) continue;
      const S sv = h ? zv.y : zv.x;
      int n;
      if constexpr (NCOUNT)   // rows without a flag hold no valid displacement and no counts
        n = (WRITE_MAP || ((fmask >> rr) & 1u)) ? nrows[(long long)yc * Wx + cx] : 0;
      else {
        // (both reads stay in row rr: an empty range reads column 0 twice)
        const bool any = lx <= hx;
        const int d1 = drow[mad24u((unsigned)rr, X1, any ? (unsigned)hx + 1 : 0u)];
        const int d0 = drow[mad24u((unsigned)rr, X1, any ? (unsigned)lx : 0u)];
        n = any ? d1 - d0 : 0;
      }
      const bool valid = n >= thr;
      const float c = valid ? (float)(sv / (S)n) : -INFINITY;
      // (zc Wy + yc < 2^24 and Wx < 2^24: a 24-bit multiply-add)
      const unsigned int canon = mad24u((unsigned)(zc * Wy + yc), Wx, (unsigned)cx);
      if (valid) {
        const unsigned long long key = ((unsigned long long)ordered_bits(c) << 32) | (0xFFFFFFFFu - canon);
        best = key > best ? key : best;
      }
      if (WRITE_MAP) {
        const long long o = ((long long)zc * Wy + yc) * Wx + cx;
        cmap[o] = c;
        if (nmap) nmap[o] = n;
      }
    }
  };
  fft_io<LC, WP, T, true, false, false>(buf, tw, pl, pack, emit);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const unsigned long long o = __shfl_xor(best, d, 64);
    best = o > best ? o : best;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = red[0];
    for (int w = 1; w < T / 64; ++w) m = red[w] > m ? red[w] : m;
    if (m) atomicMax(keys + slot, m);
  }
  };
  load_twiddles<LC>(tw, twtab, pl);
  if constexpr (WRITE_MAP) {
    // every row group, one per workgroup (a map entry is written for every displacement)
    run((int)blockIdx.z, (int)blockIdx.y, (int)blockIdx.x * NR);
  } else {
    // only the row groups that hold a valid displacement, listed by k_worklist; a fixed grid
    // strides over the list (the reduction's barrier ends each group's use of LDS)
    const unsigned n = *nwork;
    for (unsigned it = blockIdx.x; it < n; it += gridDim.x) {
      const unsigned w = work[it];
      run((int)(w >> 24), (int)((w >> 12) & 0xFFFu), (int)(w & 0xFFFu) * NR);
    }
  }
}

// ------------------------------------------------------------------------------ exact overlaps
// With a general mask on the fixed side, N(chi) is the mask cross-correlation (Sec. 3.1, after
// Eq. (5)) and no box sum gives it.  The eroded moving mask then goes through the pencil
// passes as one more field, in FP64 (k_pencil, k_zpass and k_zstore instantiated for double2)
// against A's FP64 mask spectrum, and the x C2R rounds each count to its integer: the FP64
// transform error is many orders of magnitude below the 1/2 the rounding tolerates.

// x R2C of the eroded mask: workgroup (row-pair group, interior slice z, slot).  Each pencil
// packs two interior rows as re = row y, im = row y + 1; the transform (length Px, zero
// padded) is split into the rows' half spectra with bin 0 = DC + i Nyquist and stored like
// the product fields: X1m[(z - 1)(ny - 2) + y - 1][k], k < H.
constexpr int kMaskPairs = 8;
constexpr int kThreadsM = 256;
template <int LC, bool HALF>
__global__ __launch_bounds__(kThreadsM) void k_mask_x(const uint8_t* __restrict__ mask, int nx, int ny, int nz,
                                                      long long mask_sstride, FftPlan pl,
                                                      const double2* __restrict__ twtab, double2* __restrict__ out,
                                                      int H, int Hp, long long out_sstride) {
  constexpr int W = kMaskPairs;
  extern __shared__ __align__(16) unsigned char smem[];
  const int Px = pl.L;
  double2* tw = reinterpret_cast<double2*>(smem);
  double2* buf = reinterpret_cast<double2*>(smem + align16(sizeof(double2) * Px));
  const int z = blockIdx.y + 1;
  const int slot = blockIdx.z;
  const int q0 = blockIdx.x * W;   // first row pair of this workgroup
  const int nrow = ny - 2;         // interior rows 1 .. ny - 2
  load_twiddles<LC>(tw, twtab, pl);
  if (LC == 0) __syncthreads();
  const RView m(mask + slot * mask_sstride + (long long)z * ny * nx, (long long)ny * nx);
  auto rows = [&](int i0, int i1, int p) -> double2 {
    const int x = i0 + i1;
    const int r = 2 * (q0 + p);
    const uint32_t o = (uint32_t)((1 + r) * nx + x);
    const unsigned a = m.ld1(x < nx && r < nrow ? o : kNoOff);
    const unsigned b = m.ld1(x < nx && r + 1 < nrow ? o + (uint32_t)nx : kNoOff);
    return cplx<double2>(a ? 1.0 : 0.0, b ? 1.0 : 0.0);
  };
  fft_io<LC, W, kThreadsM, false, false, true, W, HALF>(buf, tw, pl, rows, [](int, int, int, double2, int) {});
  __syncthreads();
  const RView dst(out + slot * out_sstride, 16LL * (nz - 2) * nrow * Hp);
  const uint32_t rsb = 16u * (uint32_t)Hp;
  for (int e = threadIdx.x; e < W * H; e += kThreadsM) {
    const int p = e / H, k = e - p * H;
    const double2 zk = buf[k * W + p];
    const double2 zc = buf[(k ? Px - k : Px / 2) * W + p];
    const int r = 2 * (q0 + p);
    const int row = (z - 1) * nrow + r;
    const double2 fa = k ? cplx<double2>(0.5 * (zk.x + zc.x), 0.5 * (zk.y - zc.y)) : cplx<double2>(zk.x, zc.x);
    const double2 fb = k ? cplx<double2>(0.5 * (zk.y + zc.y), 0.5 * (zc.x - zk.x)) : cplx<double2>(zk.y, zc.y);
    dst.stv<double2>(offv_if<double2>(r < nrow, row, rsb, k), fa);
    dst.stv<double2>(offv_if<double2>(r + 1 < nrow, row + 1, rsb, k), fb);
  }
}

// x C2R of the count rows (FP64) and rounding: workgroup (row group, zc, slot) as in the final
// pass, kRowsC packed row pairs Z = S1 + i S2.  Writes ncount[slot][zc][yc][cx] for the rows
// whose flag is set (all rows when every flag is set, as for a full map).
template <int LC>
__global__ __launch_bounds__(kThreadsC) void k_overlap_x(const double2* __restrict__ Y4, int* __restrict__ ncount,
                                                         int Wx, int Wy, int Wz, int H, int Hp, int x_off, FftPlan pl,
                                                         const double2* __restrict__ twtab, long long y4_sstride,
                                                         long long n_sstride, const uint8_t* __restrict__ flags,
                                                         long long flag_sstride) {
  constexpr int T = kThreadsC;
  constexpr int WP = kRowsC;
  constexpr int NR = 2 * WP;
  extern __shared__ __align__(16) unsigned char smem[];
  const int Px = pl.L;
  double2* tw = reinterpret_cast<double2*>(smem);
  double2* buf = reinterpret_cast<double2*>(smem + align16(sizeof(double2) * Px));
  const int slot = blockIdx.z, zc = blockIdx.y, yc0 = blockIdx.x * NR;
  unsigned fmask = 0;
  {
    const RView rf(flags + slot * flag_sstride + Wz + (long long)zc * Wy, Wy);   // rows >= Wy read 0
    unsigned fl[NR];
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) fl[rr] = rf.ld1((uint32_t)(yc0 + rr));
#pragma unroll
    for (int rr = 0; rr < NR; ++rr) fmask |= fl[rr] ? 1u << rr : 0u;
  }
  if (!fmask) return;
  load_twiddles<LC>(tw, twtab, pl);
  if (LC == 0) __syncthreads();
  const int half = Px / 2;
  const RView rows(Y4 + slot * y4_sstride + ((long long)zc * Wy) * Hp, 16LL * Wy * Hp);
  const uint32_t rsb = 16u * (uint32_t)Hp;
  // two rows' half spectra (bin 0 = DC + i Nyquist) as one Hermitian-extended spectrum
  auto pack = [&](int k0, int k1, int p) -> double2 {
    const int k = k0 + k1;
    const int r0 = yc0 + 2 * p;
    const bool lo = k < half;
    const int kk = k == half ? 0 : lo ? k : Px - k;
    const uint32_t o0 = offv<double2>(r0, rsb, kk);
    const double2 a = rows.ldv<double2, false>((fmask >> (2 * p)) & 1u ? o0 : kNoOff);
    const double2 c = rows.ldv<double2, false>((fmask >> (2 * p + 1)) & 1u ? o0 + rsb : kNoOff);
    const double sg = lo ? 1.0 : -1.0;
    double2 zz = cplx<double2>(fma(-sg, c.y, a.x), fma(sg, a.y, c.x));
    zz = k == 0 ? cplx<double2>(a.x, c.x) : zz;
    zz = k == half ? cplx<double2>(a.y, c.y) : zz;
    return zz;
  };
  int* out = ncount + slot * n_sstride + ((long long)zc * Wy) * Wx;
  auto emit = [&](int j0, int j1, int p, double2 zv, int) {
    int cx = j0 + j1 + x_off;   // x_off = nA_x - 1 < Px
    if (cx >= Px) cx -= Px;
    if (cx >= Wx) return;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int rr = 2 * p + h;
      const int yc = yc0 + rr;
      if (yc < Wy && ((fmask >> rr) & 1u)) out[(long long)yc * Wx + cx] = (int)rint(h ? zv.y : zv.x);
    }
  };
  fft_io<LC, WP, T, true, false, false>(buf, tw, pl, pack, emit);
}

// The final pass's work list: the (slot, zc, row group) items with any row flag set, packed
// as slot << 24 | zc << 12 | group (slots < 256, Wz and the groups < 4096).  One global atomic
// per workgroup; the order of the list is not deterministic, the results do not depend on it.
__global__ __launch_bounds__(kThreads) void k_worklist(const uint8_t* __restrict__ flags, long long flag_sstride,
                                                       int Wy, int Wz, int rows, int nslots,
                                                       unsigned* __restrict__ work, unsigned* __restrict__ nwork) {
  __shared__ unsigned cnt, base;
  const int ngroups = (Wy + rows - 1) / rows;
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  bool any = false;
  unsigned item = 0, local = 0;
  if (t < nslots * Wz * ngroups) {
    const int grp = t % ngroups, zc = (t / ngroups) % Wz, slot = t / (ngroups * Wz);
    const RView rf(flags + slot * flag_sstride + Wz + (long long)zc * Wy, Wy);   // rows >= Wy read 0
    for (int r = 0; r < rows; ++r) any |= rf.ld1((uint32_t)(grp * rows + r)) != 0;
    item = (unsigned)slot << 24 | (unsigned)zc << 12 | (unsigned)grp;
  }
  if (any) local = atomicAdd(&cnt, 1u);
  __syncthreads();
  if (threadIdx.x == 0) base = cnt ? atomicAdd(nwork, cnt) : 0u;
  __syncthreads();
  if (any) work[base + local] = item;
}

// Per-slot result from its key: score bits, canonical index -> displacement, exact N.
__global__ void k_finalize(const unsigned long long* __restrict__ keys, const int* __restrict__ sat,
                           OverlapGeom g, int Wx, int Wy, long long sat_sstride, int nslots,
                           RotResultDev* __restrict__ res, const int* __restrict__ ncount,
                           long long ncount_sstride) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nslots) return;
  const unsigned long long key = keys[slot];
  RotResultDev r;
  r.reserved = 0;
  if (key == 0ull) {
    r.score = -INFINITY;
    r.shift[0] = r.shift[1] = r.shift[2] = 0;
    r.overlap = 0;
    r.valid = 0;
  } else {
    const unsigned int hi = (unsigned int)(key >> 32);
    const unsigned int u = (hi & 0x80000000u) ? (hi & 0x7FFFFFFFu) : ~hi;
    const unsigned int canon = 0xFFFFFFFFu - (unsigned int)(key & 0xFFFFFFFFull);
    const int cx = canon % Wx, cy = (canon / Wx) % Wy, cz = canon / (Wx * Wy);
    r.score = __uint_as_float(u);
    r.shift[0] = cx - (g.nA[0] - 1);
    r.shift[1] = cy - (g.nA[1] - 1);
    r.shift[2] = cz - (g.nA[2] - 1);
    r.overlap = ncount ? (long long)ncount[slot * ncount_sstride + canon]
                       : box_count(sat + slot * sat_sstride, g, r.shift[0], r.shift[1], r.shift[2]);
    r.valid = 1;
  }
  res[slot] = r;
}

__global__ void k_fill_f32(float* __restrict__ p, long long n, float v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_check_finite(const float* __restrict__ v, long long n, int* __restrict__ flag) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  int bad = 0;
  for (; i < n; i += stride) bad |= !isfinite(v[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// ------------------------------------------------------------------------------ pyramid
// Blur taps travel by value in the kernel arguments (no device buffer): 2 K + 1 <= 513 taps,
// K = int(4 sigma + 0.5) with sigma <= 64.
constexpr int kMaxBlurTaps = 513;
struct BlurTaps {
  float w[kMaxBlurTaps];
};

// One separable pass of a Gaussian blur along one axis, keeping every step-th output sample:
// out[.., i, ..] = sum_k w[k] in[.., clamp(i * step + k - K), ..] along the axis, edges
// replicated.  in is [outer][n][inner] (the blurred axis in the middle), out is [outer][m][inner].
__global__ __launch_bounds__(kThreads) void k_blur_axis(const float* __restrict__ in, float* __restrict__ out,
                                                        int outer, int n, int inner, int m, int step,
                                                        BlurTaps taps, int K) {
  const float* w = taps.w;
  const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
  const long long total = (long long)outer * m * inner;
  if (t >= total) return;
  const int ii = (int)(t % inner);
  const int i = (int)((t / inner) % m);
  const long long o = t / ((long long)inner * m);
  const float* src = in + o * n * inner + ii;
  const int c = i * step;
  float acc = 0.f;
  for (int k = -K; k <= K; ++k) {
    int j = c + k;
    j = j < 0 ? 0 : (j >= n ? n - 1 : j);
    acc = fmaf(w[k + K], src[(long long)j * inner], acc);
  }
  out[t] = acc;
}

// Batched C2C along a contiguous axis: in/out [batch][L]; 16 batch rows per workgroup.
template <bool INV, int LC>
__global__ __launch_bounds__(kThreadsP<INV>) void k_debug_fft(const float2* __restrict__ in, float2* __restrict__ out,
                                                        int batch, FftPlan pl, const float2* __restrict__ twtab) {
  constexpr int W = kTileW;
  extern __shared__ __align__(16) unsigned char smem[];
  const int L = pl.L;
  float2* tw = reinterpret_cast<float2*>(smem);
  float2* buf = reinterpret_cast<float2*>(smem + align16(sizeof(float2) * L));
  const int b0 = blockIdx.x * W;
  load_twiddles<LC>(tw, twtab, pl);
  if (LC == 0) __syncthreads();
  fft_io<LC, W, kThreadsP<INV>, INV, false, false>(
      buf, tw, pl,
      [&](int i0, int i1, int p) -> float2 {
        return (b0 + p < batch) ? in[(long long)(b0 + p) * L + i0 + i1] : make_float2(0.f, 0.f);
      },
      [&](int k0, int k1, int p, float2 v, int) {
        if (b0 + p < batch) out[(long long)(b0 + p) * L + k0 + k1] = v;
      });
}

}  // namespace csngf
