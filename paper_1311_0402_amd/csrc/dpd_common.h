// dpd_common.h -- types and device helpers shared by the DPD kernels.
//
// Everything here is written for gfx950 (wave64).  The few functions marked
// DPD_HD are plain integer/FP arithmetic and also compile for the host, so
// the host-side library code (and a CPU unit test) can use the exact same
// cell-ranking rule as the kernels.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define DPD_HD __host__ __device__ __forceinline__
#else
#define DPD_HD inline
#endif

namespace dpd {

constexpr int kMaxTypes = 8;
constexpr int kWave = 64;
// List-build tile: two Morton-consecutive 4x4x4 cell blocks (adjacent along
// x), so a tile's cells have consecutive Morton ranks.
constexpr int kTileX = 8, kTileY = 4, kTileZ = 4;

// Kernel-side parameter block, passed by value.  Derived quantities are
// computed once on the host (inverse cell sizes, sigma / sqrt(dt), ...).
struct KParams {
    double L[3];          // box
    double halfL[3];      // L / 2 (exact)
    double inv_cell[3];   // n_c / L  (cell coordinate = trunc(x * inv_cell))
    double cell_len[3];   // L / n_c  (origin of a cell, mixed-precision offsets)
    float cell_len32[3];
    float L32[3];
    int32_t nc[3];
    int32_t nbits;        // bits of the largest cell coordinate
    int32_t n_cells;
    int32_t nb[3];        // 2x2x2 cell blocks per side (neighbour-list work units)
    int32_t nbits_b;
    int32_t n_blocks;
    int32_t small_dim[3]; // n_c < 4: a block's neighbourhood wraps onto itself
    int32_t nt[3];        // tiles of kTileX x kTileY x kTileZ cells per side (list builder)
    int32_t n_tiles;
    float tile_lo32;      // FP32 pre-test of the tile builder (tile-frame positions):
    float tile_hi32;      //   r^2 < lo is a neighbour, r^2 >= hi is not, else FP64 decides
    float list_lo32;      // FP32 pre-test: r^2 < lo is a neighbour for sure,
    float list_hi32;      // r^2 >= hi is not; in between the FP64 test decides
    double rl2;           // (r_c + skin)^2, neighbour test  r^2 < rl2
    double rc2;           // r_c^2, force test              r^2 < rc2
    double r_c;
    double inv_rc;
    double dt;
    double half_dt;
    double lam_dt;        // lambda * dt
    int32_t lam_half;     // lambda == 1/2: predicted velocity is the half-step one
    int32_t wmode;        // w_R = w_C^s: 0 = sqrt, 1 = w_C, 2 = w_C^2, 3 = pow
    double s;
    int32_t n_types;
    uint32_t seed_lo, seed_hi;
    double body_g, body_split;
    double bond_k, bond_r0;
    const int32_t* partner;     // device, by tag; nullptr = no bonds
    // position of this system inside a batch (all 0 for a single system)
    int32_t p_off, c_off, b_off, n_local;
    int32_t t_off;
    // per type pair: a, gamma, sigma / sqrt(dt)
    double a[kMaxTypes * kMaxTypes];
    double g[kMaxTypes * kMaxTypes];
    double srdt[kMaxTypes * kMaxTypes];
};

// ---------------------------------------------------------------------------
// Morton rank of a cell on an n_x x n_y x n_z grid, computed by counting:
// rank(c) = number of grid cells whose Morton code (bit b of x at 3b, of y
// at 3b+1, of z at 3b+2) is smaller than c's.  Walking the code from its most
// significant bit, every 1-bit of c adds the number of grid cells that share
// c's higher bits and have a 0 there; that number factorises into one count
// per axis of the integers in [0, n) with a given high-bit prefix.
// ---------------------------------------------------------------------------

DPD_HD int64_t prefix_count(int64_t prefix, int shift, int64_t n)
{
    // integers v in [0, n) with (v >> shift) == prefix
    int64_t lo = prefix << shift;
    int64_t hi = (prefix + 1) << shift;
    if (hi > n) hi = n;
    return hi > lo ? hi - lo : 0;
}

DPD_HD int32_t morton_rank(int32_t cx, int32_t cy, int32_t cz,
                           int32_t nx, int32_t ny, int32_t nz, int32_t nbits)
{
    int64_t rank = 0;
    int64_t px = 0, py = 0, pz = 0;  // high bits fixed so far, per axis
    for (int b = nbits - 1; b >= 0; --b) {
        const int bz = (cz >> b) & 1;
        if (bz) rank += prefix_count(2 * pz, b, nz) * prefix_count(py, b + 1, ny) * prefix_count(px, b + 1, nx);
        pz = 2 * pz + bz;
        const int by = (cy >> b) & 1;
        if (by) rank += prefix_count(pz, b, nz) * prefix_count(2 * py, b, ny) * prefix_count(px, b + 1, nx);
        py = 2 * py + by;
        const int bx = (cx >> b) & 1;
        if (bx) rank += prefix_count(pz, b, nz) * prefix_count(py, b, ny) * prefix_count(2 * px, b, nx);
        px = 2 * px + bx;
    }
    return (int32_t)rank;
}

// Inverse of morton_rank: the cell whose rank is r (0 <= r < nx*ny*nz).
// Same walk; at every code bit, a 0 is taken while r is below the number
// of grid cells with that prefix, otherwise r drops by that number.
DPD_HD void morton_unrank(int64_t r, int32_t nx, int32_t ny, int32_t nz, int32_t nbits,
                          int32_t* cx, int32_t* cy, int32_t* cz)
{
    int64_t px = 0, py = 0, pz = 0;
    for (int b = nbits - 1; b >= 0; --b) {
        int64_t c0 = prefix_count(2 * pz, b, nz) * prefix_count(py, b + 1, ny) * prefix_count(px, b + 1, nx);
        int bz = 0;
        if (r >= c0) { r -= c0; bz = 1; }
        pz = 2 * pz + bz;
        c0 = prefix_count(pz, b, nz) * prefix_count(2 * py, b, ny) * prefix_count(px, b + 1, nx);
        int by = 0;
        if (r >= c0) { r -= c0; by = 1; }
        py = 2 * py + by;
        c0 = prefix_count(pz, b, nz) * prefix_count(py, b, ny) * prefix_count(2 * px, b, nx);
        int bx = 0;
        if (r >= c0) { r -= c0; bx = 1; }
        px = 2 * px + bx;
    }
    *cx = (int32_t)px;
    *cy = (int32_t)py;
    *cz = (int32_t)pz;
}

DPD_HD int32_t bits_for(int32_t nmax)
{
    int32_t b = 1;
    while ((1 << b) < nmax) ++b;
    return b;
}

// Batcher's odd-even merge sorting network for n <= 64 keys, built at
// compile time (iterative form: runs of length p are merged by comparators
// k apart, k = p, p/2, ..., 1).  Comparator c orders keys a[c] < b[c].
struct SortNet {
    int count;
    unsigned char a[512], b[512];
};

constexpr SortNet make_sort_net(int n)
{
    SortNet net{};
    net.count = 0;
    for (int p = 1; p < n; p <<= 1)
        for (int k = p; k >= 1; k >>= 1)
            for (int j = k % p; j <= n - 1 - k; j += 2 * k)
                for (int i = 0; i <= (k - 1 < n - j - k - 1 ? k - 1 : n - j - k - 1); ++i)
                    if ((i + j) / (2 * p) == (i + j + k) / (2 * p)) {
                        net.a[net.count] = (unsigned char)(i + j);
                        net.b[net.count] = (unsigned char)(i + j + k);
                        ++net.count;
                    }
    return net;
}

DPD_HD uint32_t pack_cell(int32_t cx, int32_t cy, int32_t cz)
{
    return (uint32_t)cx | ((uint32_t)cy << 10) | ((uint32_t)cz << 20);
}

// A gate: a kernel given one does its work only while *gate != 0 (a null
// gate always lets it run).  With a Verlet skin, dpd_step sets the gate of
// every step from the particles' displacements since the last rebuild, and
// the kernels of binning, reordering and the list build read it (whole
// blocks leave at once, so no barrier is skipped by part of a block).
using Gate = const int32_t*;

// A batch of independent systems: one KParams per system in device memory,
// particle / cell / list-block offsets (n_sys + 1 entries each) and the
// static particle -> system map.  kps == nullptr means a single system.
struct BatchView {
    const KParams* kps;
    const int32_t* p_off;
    const int32_t* c_off;
    const int32_t* b_off;
    const int32_t* t_off;    // list-build tiles, numbered system by system
    const int32_t* ch_off;   // 64-row force chunks, numbered system by system
    const uint16_t* sys_of;
    int32_t n_sys;
    int32_t n_chunks;        // ch_off[n_sys]
};

#if defined(__HIPCC__)

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool gated_off(Gate g) { return g != nullptr && *g == 0; }

// largest s in [0, n_seg) with off[s] <= x (off ascending)
__device__ __forceinline__ int32_t find_segment(const int32_t* __restrict__ off, int32_t n_seg, int32_t x)
{
    int32_t lo = 0, hi = n_seg;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// Workgroups are dealt to the 8 XCDs round-robin; renumber them so every
// XCD (and its L2) works through one contiguous range of logical ids.
__device__ __forceinline__ int32_t xcd_logical_id(int32_t p, int32_t groups)
{
    const int32_t q = groups / 8, r = groups % 8;
    const int32_t xcd = p % 8, k = p / 8;
    return xcd < r ? xcd * (q + 1) + k : r * (q + 1) + (xcd - r) * q + k;
}

// ---------------------------------------------------------------------------
// (continued) device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// number of set bits of `mask` in lanes below this one
__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int32_t cell_coord(double x, double inv_cell, int32_t n)
{
    // truncation of x n_c / L, clamped to [0, n - 1] before the conversion
    // (the same cell as clamping after it, since n - 1 is an integer); a
    // non-finite position lands in cell 0 instead of an undefined integer
    double q = x * inv_cell;
    q = q > 0.0 ? q : 0.0;
    q = q < (double)(n - 1) ? q : (double)(n - 1);
    return (int32_t)q;
}

__device__ __forceinline__ double min_image(double d, double L, double halfL)
{
    // subtract first, then shift by one box length (no pre-shifted copies)
    if (d > halfL) d = d - L;
    else if (d < -halfL) d = d + L;
    return d;
}

__device__ __forceinline__ double dist2(double dx, double dy, double dz)
{
    return __fma_rn(dz, dz, __fma_rn(dy, dy, __dmul_rn(dx, dx)));
}

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies and xors, key bumped by the Weyl constants.  Each
// multiply is written as one 64-bit product so it maps to a single
// v_mad_u64_u32 (high and low word together).
struct U4 { uint32_t x, y, z, w; };

// a ^ b ^ c in one v_bitop3_b32 (truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = U4{xor3((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1, xor3((uint32_t)(p0 >> 32), c.w, k1), (uint32_t)p0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ U4 pair_words(uint32_t ti, uint32_t tj, uint64_t step,
                                         uint32_t seed_lo, uint32_t seed_hi)
{
    const uint32_t a = ti < tj ? ti : tj;
    const uint32_t b = ti < tj ? tj : ti;
    return philox4x32_10(U4{a, b, (uint32_t)step, (uint32_t)(step >> 32)}, seed_lo, seed_hi);
}

// xi = sqrt(-2 ln u1) cos(2 pi u2), u1 = (w0 + 1/2) 2^-32, u2 = w1 2^-32 (FP64)
__device__ __forceinline__ double gauss64(U4 w)
{
    const double u1 = ((double)w.x + 0.5) * 0x1p-32;
    const double u2 = (double)w.y * 0x1p-32;
    return sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

// Same variate in FP32 with the hardware transcendentals: v_log_f32 (log2),
// v_cos_f32 (argument in revolutions, so cos(2 pi u2) is one instruction) and
// v_sqrt_f32.  For w0 >= 2^31, u1 is close to 1 and rounding u1 itself
// would dominate ln(u1); there ln(u1) = ln(1 - t) with the complement
// t = (2^32 - 1 - w0 + 1/2) 2^-32 formed in integers first: a four-term
// series for t < 2^-7, log2(1 - t) above.
__device__ __forceinline__ float gauss32(U4 w)
{
    constexpr float kLn2 = 0.693147180559945309f;
    // (w + 1/2) 2^-32 as one fused multiply-add on the converted word
    const float u1 = __fmaf_rn((float)w.x, 0x1p-32f, 0x1p-33f);
    const float t = __fmaf_rn((float)(0xFFFFFFFFu - w.x), 0x1p-32f, 0x1p-33f);
    const float series = -t * __fmaf_rn(t, __fmaf_rn(t, __fmaf_rn(t, 0.25f, 0.333333333f), 0.5f), 1.0f);
    const float lg = __builtin_amdgcn_logf(w.x >= 0x80000000u ? 1.0f - t : u1) * kLn2;
    const float lnu = (w.x >= 0x80000000u && t < 0x1p-7f) ? series : lg;
    const float u2 = (float)w.y * 0x1p-32f;
    return __builtin_amdgcn_sqrtf(-2.0f * lnu) * __builtin_amdgcn_cosf(u2);
}

#endif  // __HIPCC__

}  // namespace dpd
