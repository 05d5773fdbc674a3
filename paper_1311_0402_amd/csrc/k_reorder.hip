// k_reorder.hip -- cell binning, device-wide scan and particle reordering
// (Sec. 3.2.2 / 3.2.3 of the paper: particles of one cell get consecutive
// indices, cells follow a Morton curve; here the order inside a cell is by
// tag, which makes the permutation a deterministic total order).
//
// Pipeline: k_bin (cell rank + slot by atomic count) -> exclusive scan of
// the counts (= cell_start) -> k_place (scatter to count slots) ->
// k_finalize (rank by tag inside the cell, gather all particle arrays).
// The atomics only decide provisional slots; the final position depends on
// (cell rank, tag) alone.
#include "dpd_launch.h"

namespace dpd {

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t count, int32_t value, Gate gate)
{
    if (gated_off(gate)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

__global__ void k_zero3(int32_t* __restrict__ a, int32_t* __restrict__ b, int32_t* __restrict__ c, Gate gate)
{
    if (gated_off(gate)) return;
    if (threadIdx.x == 0 && a) *a = 0;
    if (threadIdx.x == 1 && b) *b = 0;
    if (threadIdx.x == 2 && c) *c = 0;
}

hipError_t launch_zero3(int32_t* a, int32_t* b, int32_t* c, hipStream_t s, Gate gate)
{
    hipLaunchKernelGGL(k_zero3, dim3(1), dim3(kWave), 0, s, a, b, c, gate);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t value, hipStream_t s, Gate gate)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(ceil_div(count, kBlock)), dim3(kBlock), 0, s, p, count, value, gate);
    return hipGetLastError();
}

// Morton rank of every cell; in a batch the table covers all systems' cells
// (system s at c_off[s]) and holds global ranks c_off[s] + local rank.
__device__ __forceinline__ void rank_one(const KParams& P, int32_t* __restrict__ rank_tab, int32_t c)
{
    const int32_t lc = c - P.c_off;
    const int32_t cx = lc % P.nc[0];
    const int32_t cy = (lc / P.nc[0]) % P.nc[1];
    const int32_t cz = lc / (P.nc[0] * P.nc[1]);
    rank_tab[c] = P.c_off + morton_rank(cx, cy, cz, P.nc[0], P.nc[1], P.nc[2], P.nbits);
}

template <bool kB>
__global__ __launch_bounds__(kBlock) void k_rank_table(KParams kp, BatchView bv, int32_t c_tot,
                                                       int32_t* __restrict__ rank_tab)
{
    const int32_t c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= c_tot) return;
    if constexpr (kB) rank_one(bv.kps[find_segment(bv.c_off, bv.n_sys, c)], rank_tab, c);
    else rank_one(kp, rank_tab, c);
}

hipError_t launch_rank_table(const KParams& kp, const BatchView& bv, int32_t c_tot, int32_t* rank_tab,
                             hipStream_t s)
{
    if (c_tot <= 0) return hipSuccess;
    if (bv.kps)
        hipLaunchKernelGGL(k_rank_table<true>, dim3(ceil_div(c_tot, kBlock)), dim3(kBlock), 0, s, kp, bv, c_tot,
                           rank_tab);
    else
        hipLaunchKernelGGL(k_rank_table<false>, dim3(ceil_div(c_tot, kBlock)), dim3(kBlock), 0, s, kp, bv, c_tot,
                           rank_tab);
    return hipGetLastError();
}

__device__ __forceinline__ int32_t bin_one(const KParams& P, int32_t n, int32_t i, const double* __restrict__ x,
                                           const int32_t* __restrict__ rank_tab, int32_t* __restrict__ key,
                                           uint32_t* __restrict__ cxyz)
{
    const int32_t cx = cell_coord(x[i], P.inv_cell[0], P.nc[0]);
    const int32_t cy = cell_coord(x[(int64_t)n + i], P.inv_cell[1], P.nc[1]);
    const int32_t cz = cell_coord(x[2 * (int64_t)n + i], P.inv_cell[2], P.nc[2]);
    const int32_t r = rank_tab[P.c_off + cx + P.nc[0] * (cy + P.nc[1] * cz)];
    key[i] = r;
    cxyz[i] = pack_cell(cx, cy, cz);
    return r;
}

// Cell of every particle and a provisional slot inside it.  The state comes
// in nearly sorted (last step's order), so neighbouring lanes mostly share a
// cell: each run of equal keys in consecutive lanes takes its slots with one
// atomic.  Slots only need to be distinct; the final in-cell order is by tag.
template <bool kB>
__global__ __launch_bounds__(kBlock) void k_bin(KParams kp, BatchView bv, int32_t n, const double* __restrict__ x,
                                                const int32_t* __restrict__ rank_tab,
                                                int32_t* __restrict__ key, int32_t* __restrict__ slot,
                                                uint32_t* __restrict__ cxyz, int32_t* __restrict__ counts,
                                                Gate gate)
{
    if (gated_off(gate)) return;
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    const bool live = i < n;
    int32_t r = -1;
    if (live) {
        if constexpr (kB) r = bin_one(bv.kps[bv.sys_of[i]], n, i, x, rank_tab, key, cxyz);
        else r = bin_one(kp, n, i, x, rank_tab, key, cxyz);
    }
    const int lane = (int)lane_id();
    const int32_t prev = __shfl_up(r, 1, kWave);
    const bool head = live && (lane == 0 || prev != r);
    // live lanes are a prefix of the wave; the first dead lane ends the last run
    const uint64_t bounds = __ballot(head) | ~__ballot(live);
    const uint64_t le = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull);
    const int start = 63 - __clzll(bounds & le);
    const uint64_t after = bounds & ~le;
    const int end = after ? __ffsll((long long)after) - 1 : kWave;
    int32_t base = 0;
    if (head) base = atomicAdd(&counts[r], end - start);
    base = __shfl(base, start, kWave);
    if (live) slot[i] = base + (lane - start);
}

hipError_t launch_bin(const KParams& kp, const BatchView& bv, int32_t n, const double* x, const int32_t* rank_tab,
                      int32_t* key, int32_t* slot, uint32_t* cxyz, int32_t* counts, hipStream_t s, Gate gate)
{
    if (n <= 0) return hipSuccess;
    if (bv.kps)
        hipLaunchKernelGGL(k_bin<true>, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, kp, bv, n, x, rank_tab, key,
                           slot, cxyz, counts, gate);
    else
        hipLaunchKernelGGL(k_bin<false>, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, kp, bv, n, x, rank_tab, key,
                           slot, cxyz, counts, gate);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan (three passes: tile sums, scan of the tile
// sums, tile-local scan plus tile offset).  Tiles of kScanTile items, 256
// threads x 16 items, wave64 shuffles inside a wave.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int32_t wave_incl_scan(int32_t v)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

// exclusive scan of one value per thread over the block; *total = block sum
__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t* s_wave, int32_t* total)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    const int32_t incl = wave_incl_scan(v);
    if (lane == kWave - 1) s_wave[w] = incl;
    __syncthreads();
    int32_t off = 0, tot = 0;
    for (int k = 0; k < nw; ++k) {
        const int32_t t = s_wave[k];
        off += (k < w) ? t : 0;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_tiles(const int32_t* __restrict__ data, int64_t count,
                                                       int32_t* __restrict__ partials, Gate gate)
{
    if (gated_off(gate)) return;
    __shared__ int32_t s_wave[kBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int32_t sum = 0;
    if (base + kScanTile <= count && (reinterpret_cast<uintptr_t>(data) & 15) == 0) {
        // a whole tile: its items as int4 loads, all issued at once
        const int4* __restrict__ p = reinterpret_cast<const int4*>(data + base);
#pragma unroll
        for (int q = 0; q < kScanTile / 4 / kBlock; ++q) {
            const int4 v = p[threadIdx.x + q * kBlock];
            sum += (v.x + v.y) + (v.z + v.w);
        }
    } else {
        for (int k = threadIdx.x; k < kScanTile; k += kBlock) {
            const int64_t i = base + k;
            if (i < count) sum += data[i];
        }
    }
    int32_t tot;
    block_excl_scan(sum, s_wave, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_partials(int32_t* __restrict__ partials, int32_t n_tiles, Gate gate)
{
    if (gated_off(gate)) return;
    __shared__ int32_t s_wave[1024 / kWave];
    int32_t carry = 0;
    for (int32_t base = 0; base < n_tiles; base += 1024) {
        const int32_t i = base + threadIdx.x;
        const int32_t v = i < n_tiles ? partials[i] : 0;
        int32_t tot;
        const int32_t ex = block_excl_scan(v, s_wave, &tot);
        if (i < n_tiles) partials[i] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(int32_t* __restrict__ data, int64_t count,
                                                       const int32_t* __restrict__ partials, Gate gate)
{
    if (gated_off(gate)) return;
    constexpr int kItems = kScanTile / kBlock;   // 16
    // +1 padding per 16 items so the per-thread runs do not share banks
    __shared__ int32_t s_tile[kScanTile + kScanTile / kItems];
    __shared__ int32_t s_wave[kBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const bool whole = base + kScanTile <= count && (reinterpret_cast<uintptr_t>(data) & 15) == 0;
    if (whole) {
        const int4* __restrict__ p = reinterpret_cast<const int4*>(data + base);
#pragma unroll
        for (int q = 0; q < kScanTile / 4 / kBlock; ++q) {
            const int k = 4 * (threadIdx.x + q * kBlock);     // 4 items of one 16-item run
            const int4 v = p[threadIdx.x + q * kBlock];
            const int a = k + k / kItems;
            s_tile[a] = v.x; s_tile[a + 1] = v.y; s_tile[a + 2] = v.z; s_tile[a + 3] = v.w;
        }
    } else {
        for (int k = threadIdx.x; k < kScanTile; k += kBlock) {
            const int64_t i = base + k;
            s_tile[k + k / kItems] = i < count ? data[i] : 0;
        }
    }
    __syncthreads();
    const int t0 = threadIdx.x * kItems;
    int32_t run = 0;
#pragma unroll
    for (int q = 0; q < kItems; ++q) run += s_tile[t0 + q + (t0 + q) / kItems];
    int32_t tot;
    int32_t ex = block_excl_scan(run, s_wave, &tot) + partials[blockIdx.x];
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
        const int a = t0 + q + (t0 + q) / kItems;
        const int32_t v = s_tile[a];
        s_tile[a] = ex;
        ex += v;
    }
    __syncthreads();
    if (whole) {
        int4* __restrict__ p = reinterpret_cast<int4*>(data + base);
#pragma unroll
        for (int q = 0; q < kScanTile / 4 / kBlock; ++q) {
            const int k = 4 * (threadIdx.x + q * kBlock);
            const int a = k + k / kItems;
            p[threadIdx.x + q * kBlock] = make_int4(s_tile[a], s_tile[a + 1], s_tile[a + 2], s_tile[a + 3]);
        }
    } else {
        for (int k = threadIdx.x; k < kScanTile; k += kBlock) {
            const int64_t i = base + k;
            if (i < count) data[i] = s_tile[k + k / kItems];
        }
    }
}

hipError_t launch_scan(int32_t* data, int64_t count, int32_t* partials, hipStream_t s, Gate gate)
{
    if (count <= 0) return hipSuccess;
    const int tiles = ceil_div(count, kScanTile);
    hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kBlock), 0, s, data, count, partials, gate);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partials, tiles, gate);
    hipLaunchKernelGGL(k_scan_apply, dim3(tiles), dim3(kBlock), 0, s, data, count, partials, gate);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scatter into provisional slots, then the final (cell rank, tag) order.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_place(int32_t n, const int32_t* __restrict__ key,
                                                  const int32_t* __restrict__ slot,
                                                  const int32_t* __restrict__ cell_start,
                                                  const uint32_t* __restrict__ tag,
                                                  uint32_t* __restrict__ tmp_tag, int32_t* __restrict__ tmp_src,
                                                  int32_t* __restrict__ tmp_key, Gate gate)
{
    if (gated_off(gate)) return;
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t k = key[i];
    const int32_t pos = cell_start[k] + slot[i];
    tmp_tag[pos] = tag[i];
    tmp_src[pos] = i;
    tmp_key[pos] = k;
}

hipError_t launch_place(int32_t n, const int32_t* key, const int32_t* slot, const int32_t* cell_start,
                        const uint32_t* tag, uint32_t* tmp_tag, int32_t* tmp_src, int32_t* tmp_key, hipStream_t s,
                        Gate gate)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_place, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, n, key, slot, cell_start,
                       tag, tmp_tag, tmp_src, tmp_key, gate);
    return hipGetLastError();
}

__device__ __forceinline__ void finalize_one(const KParams& P, int32_t n, int32_t p,
                                             const int32_t* __restrict__ tmp_key,
                                             const int32_t* __restrict__ cell_start,
                                             const uint32_t* __restrict__ tmp_tag,
                                             const int32_t* __restrict__ tmp_src, const GatherArgs& g)
{
    // everything that depends only on the source is requested before the
    // in-cell rank (which needs the cell's bounds and tags)
    const int32_t src = tmp_src[p];
    const int32_t c = tmp_key[p];
    const uint32_t t = tmp_tag[p];
    const int64_t N = n;
    double xs[3], vs[3], vts[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        xs[k] = g.x_in[k * N + src];
        vs[k] = g.v_in[k * N + src];
        vts[k] = g.vt_in ? g.vt_in[k * N + src] : 0.0;
    }
    const uint8_t ty = g.type_in[src];
    const uint32_t packed = g.cxyz_in[src];
    const int32_t lo = cell_start[c], hi = cell_start[c + 1];
    // the cell's first four tags are requested together (most cells hold
    // fewer; reads past the last particle stay inside the array)
    int32_t below = 0;
    uint32_t t4[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) t4[m] = tmp_tag[lo + m < n ? lo + m : n - 1];
#pragma unroll
    for (int m = 0; m < 4; ++m) below += (lo + m < hi && t4[m] < t) ? 1 : 0;
    for (int32_t q = lo + 4; q < hi; ++q) below += (tmp_tag[q] < t) ? 1 : 0;
    const int32_t dst = lo + below;
    g.perm[dst] = src;
    if (g.inv) g.inv[src] = dst;
    g.tag_out[dst] = t;
    g.type_out[dst] = ty;
    g.cell_xyz[dst] = packed;
    // tags are numbered per system (0 .. n_local - 1)
    const uint32_t n_tags = (uint32_t)(P.n_local > 0 ? P.n_local : n);
    if (g.idx_of_tag && t < n_tags) g.idx_of_tag[P.p_off + t] = dst;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        g.x_out[k * N + dst] = xs[k];
        g.v_out[k * N + dst] = vs[k];
    }
    if (g.xref) {
#pragma unroll
        for (int k = 0; k < 3; ++k) g.xref[k * N + dst] = xs[k];
    }
    if (g.vt_in) {
#pragma unroll
        for (int k = 0; k < 3; ++k) g.vt_out[k * N + dst] = vts[k];
    }
    if (g.x32) {
        const int32_t cc[3] = {(int32_t)(packed & 1023u), (int32_t)((packed >> 10) & 1023u),
                               (int32_t)(packed >> 20)};
        float4 w;
        w.x = (float)(xs[0] - (double)cc[0] * P.cell_len[0]);
        w.y = (float)(xs[1] - (double)cc[1] * P.cell_len[1]);
        w.z = (float)(xs[2] - (double)cc[2] * P.cell_len[2]);
        w.w = __uint_as_float(t);
        reinterpret_cast<float4*>(g.x32)[dst] = w;
    }
    if (g.x64) {
        // packed FP64 copies for the FP64 force pass: position and tag, the
        // velocity the forces see and the type
        const double* vv = g.vt_in ? vts : vs;
        double4 px, pv;
        px.x = xs[0]; px.y = xs[1]; px.z = xs[2]; px.w = __longlong_as_double((long long)t);
        pv.x = vv[0]; pv.y = vv[1]; pv.z = vv[2]; pv.w = __longlong_as_double((long long)ty);
        reinterpret_cast<double4*>(g.x64)[dst] = px;
        reinterpret_cast<double4*>(g.v64)[dst] = pv;
    }
    if (g.v32) {
        // the predicted velocity: v~ when it is kept apart, else v
        const double* vv = g.vt_in ? vts : vs;
        float4 w;
        w.x = (float)vv[0];
        w.y = (float)vv[1];
        w.z = (float)vv[2];
        w.w = __uint_as_float((uint32_t)ty);
        reinterpret_cast<float4*>(g.v32)[dst] = w;
    }
}

template <bool kB>
__global__ __launch_bounds__(kBlock) void k_finalize(KParams kp, BatchView bv, int32_t n,
                                                     const int32_t* __restrict__ tmp_key,
                                                     const int32_t* __restrict__ cell_start,
                                                     const uint32_t* __restrict__ tmp_tag,
                                                     const int32_t* __restrict__ tmp_src, GatherArgs g, Gate gate)
{
    if (gated_off(gate)) return;
    const int32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    // a particle never leaves its system, so position p and its source share it
    if constexpr (kB) finalize_one(bv.kps[bv.sys_of[p]], n, p, tmp_key, cell_start, tmp_tag, tmp_src, g);
    else finalize_one(kp, n, p, tmp_key, cell_start, tmp_tag, tmp_src, g);
}

namespace {

__global__ __launch_bounds__(kBlock) void k_pidx_init(int32_t n, const uint32_t* __restrict__ tag,
                                                      const int32_t* __restrict__ partner, int32_t n_tags,
                                                      const int32_t* __restrict__ idx_of_tag,
                                                      int32_t* __restrict__ pidx)
{
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t t = tag[i];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        int32_t j = -1;
        if (t < (uint32_t)n_tags) {
            const int32_t pt = partner[2 * (int64_t)t + b];
            if (pt >= 0) {
                j = pt < n_tags ? idx_of_tag[pt] : -2;
                j = (j >= 0 && j < n) ? j : -2;
            }
        }
        pidx[2 * (int64_t)i + b] = j;
    }
}

__global__ __launch_bounds__(kBlock) void k_pidx_update(int32_t n, const int32_t* __restrict__ perm,
                                                        const int32_t* __restrict__ inv,
                                                        const int32_t* __restrict__ pidx_old,
                                                        int32_t* __restrict__ pidx_new, Gate gate)
{
    const int32_t d = blockIdx.x * kBlock + threadIdx.x;
    if (d >= n) return;
    if (gated_off(gate)) {
        // no reorder this step: the indices carry over unchanged
        reinterpret_cast<int2*>(pidx_new)[d] = reinterpret_cast<const int2*>(pidx_old)[d];
        return;
    }
    const int32_t src = perm[d];
    // a particle's two partners as one 8-byte access (the arrays are
    // 8-byte aligned workspace)
    const int2 po = reinterpret_cast<const int2*>(pidx_old)[src];
    int2 pn;
    pn.x = po.x < 0 ? po.x : inv[po.x];
    pn.y = po.y < 0 ? po.y : inv[po.y];
    reinterpret_cast<int2*>(pidx_new)[d] = pn;
}

}  // namespace

hipError_t launch_pidx_init(const KParams& kp, int32_t n, const uint32_t* tag, const int32_t* idx_of_tag,
                            int32_t* pidx, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    // tags of a single system run 0 .. n - 1
    hipLaunchKernelGGL(k_pidx_init, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, n, tag, kp.partner, n,
                       idx_of_tag, pidx);
    return hipGetLastError();
}

hipError_t launch_pidx_update(int32_t n, const int32_t* perm, const int32_t* inv, const int32_t* pidx_old,
                              int32_t* pidx_new, hipStream_t s, Gate gate)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pidx_update, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, n, perm, inv, pidx_old,
                       pidx_new, gate);
    return hipGetLastError();
}

namespace {

__global__ __launch_bounds__(kBlock) void k_precopy(int32_t n, const double* __restrict__ x,
                                                    const double* __restrict__ v, const double* __restrict__ vt,
                                                    const uint32_t* __restrict__ tag,
                                                    const uint8_t* __restrict__ type, double* __restrict__ bx,
                                                    double* __restrict__ bv, double* __restrict__ bvt,
                                                    uint32_t* __restrict__ btag, uint8_t* __restrict__ btype,
                                                    Gate gate)
{
    if (gated_off(gate)) return;
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t N = n;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        bx[k * N + i] = x[k * N + i];
        bv[k * N + i] = v[k * N + i];
        if (vt) bvt[k * N + i] = vt[k * N + i];
    }
    btag[i] = tag[i];
    btype[i] = type[i];
}

}  // namespace

hipError_t launch_precopy(int32_t n, const double* x, const double* v, const double* vt, const uint32_t* tag,
                          const uint8_t* type, double* bx, double* bv, double* bvt, uint32_t* btag,
                          uint8_t* btype, hipStream_t s, Gate gate)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_precopy, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, n, x, v, vt, tag, type, bx, bv,
                       bvt, btag, btype, gate);
    return hipGetLastError();
}

hipError_t launch_finalize(const KParams& kp, const BatchView& bv, int32_t n, const int32_t* tmp_key,
                           const int32_t* cell_start, const uint32_t* tmp_tag, const int32_t* tmp_src,
                           const GatherArgs& g, hipStream_t s, Gate gate)
{
    if (n <= 0) return hipSuccess;
    if (bv.kps)
        hipLaunchKernelGGL(k_finalize<true>, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, kp, bv, n, tmp_key,
                           cell_start, tmp_tag, tmp_src, g, gate);
    else
        hipLaunchKernelGGL(k_finalize<false>, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, kp, bv, n, tmp_key,
                           cell_start, tmp_tag, tmp_src, g, gate);
    return hipGetLastError();
}

}  // namespace dpd
