// k_nlist.hip -- ordered neighbour list (Sec. 3.3 of the paper).
//
// Work unit: one 64-lane wavefront per Morton-aligned 2x2x2 block of cells.
// The block's cells have consecutive Morton ranks, so its particles (the i
// side) are one contiguous index range.  The union of their stencils is the
// 4x4x4 cells around the block (fewer where a side has only 3 cells); lane m
// takes union cell m, the cells are put in ascending rank (each lane counts
// the smaller ranks, then pushes its data to that lane with ds_permute) and
// their particle ranges concatenate into one strictly ascending candidate
// sequence, as the paper's sorted stencil does.  Lanes walk the candidates 64
// at a time; for every particle i of the block the wave ballots the distance
// test and a hit's slot in i's row is the row's running count plus the hits
// in lower lanes (mbcnt).  Rows are ascending and deterministic, no atomics.
//
// Distance test: separations in FP32 from the particles' offsets inside their
// cells plus whole-cell offsets in the block frame.  Outside a narrow band
// around r_list^2 the FP32 value decides; inside it the exact FP64 rule
// (minimum image, fma order) decides, so the rows equal the FP64 definition
// bit for bit.  Candidates two cells away from i fail the test (cells are
// wider than r_list).
//
// One pass writes every row into a fixed-width scratch slab and the row
// sizes; a scan makes the CSR offsets and a compaction copies the rows into
// the CSR list.  Rows that do not fit the slab width send the build through
// a second, direct pass instead (same walk, writing at the scanned offsets).
//
// Second work unit (the default while all ranks fit 27 bits): one lane per
// particle i.  The lane ranks i's 27 stencil cells, sorts them by rank with
// a fixed comparison network (Batcher's odd-even merge sort), and walks them
// in that order, each cell's particles in index order, so its row comes out
// ascending with no cross-lane work.  Lanes of a wave walk their own k-th
// stencil cells together; the distance test is the same FP32 pre-test with
// the same exact FP64 band rule.
#include <climits>
#include <cmath>

#include "dpd_launch.h"

namespace dpd {

namespace {

constexpr int kWavesPerBlock = kBlock / kWave;

__device__ __forceinline__ int32_t wrap_cell(int32_t c, int32_t n)
{
    c = c < 0 ? c + n : c;
    return c >= n ? c - n : c;
}

// index into the (batch-wide) rank table
__device__ __forceinline__ int32_t lin_cell(const KParams& kp, int32_t cx, int32_t cy, int32_t cz)
{
    return kp.c_off + cx + kp.nc[0] * (cy + kp.nc[1] * cz);
}

__device__ __forceinline__ float min_image32(float d, float L)
{
    const float h = 0.5f * L;
    d = d > h ? d - L : d;
    return d < -h ? d + L : d;
}

// exact FP64 neighbour rule for one pair (same operations as everywhere else)
__device__ __forceinline__ bool exact_hit(const KParams& kp, const double* __restrict__ x, int64_t N,
                                          int32_t i, int32_t j)
{
    const double dx = min_image(x[i] - x[j], kp.L[0], kp.halfL[0]);
    const double dy = min_image(x[N + i] - x[N + j], kp.L[1], kp.halfL[1]);
    const double dz = min_image(x[2 * N + i] - x[2 * N + j], kp.L[2], kp.halfL[2]);
    return dist2(dx, dy, dz) < kp.rl2;
}

// kDirect = false: rows go to a fixed-width scratch slab (row i at
// slab[i * K]) and row sizes to offset[]; a scan and k_nlist_compact then
// produce the CSR list.  kDirect = true: the same walk writes straight into
// the CSR list (needs the scanned offsets); it only runs when some row did
// not fit its K slab slots.
template <bool kDirect>
__device__ __forceinline__ void nlist_block(const KParams& kp, int32_t blk, int32_t n,
                                            const double* __restrict__ x, const float* __restrict__ x32,
                                            const int32_t* __restrict__ cell_start,
                                            const int32_t* __restrict__ rank_tab, int32_t* __restrict__ offset,
                                            int32_t* __restrict__ index, int32_t* __restrict__ slab,
                                            int32_t slab_k, int32_t* __restrict__ flag)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t N = n;

    // ---- the block and its particle range ----
    int32_t bx, by, bz;
    morton_unrank(blk, kp.nb[0], kp.nb[1], kp.nb[2], kp.nbits_b, &bx, &by, &bz);
    const int32_t o[3] = {2 * bx, 2 * by, 2 * bz};                 // block origin (cells)
    int32_t vd[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) vd[d] = (kp.nc[d] - o[d] >= 2) ? 2 : 1;
    const int32_t nv = vd[0] * vd[1] * vd[2];
    const int32_t r0 = rank_tab[lin_cell(kp, o[0], o[1], o[2])];
    const int32_t i_lo = cell_start[r0], i_hi = cell_start[r0 + nv];
    if (i_lo == i_hi) return;

    // ---- union of the block's stencils: lane m < U owns union cell m ----
    int32_t ulo[3], ucnt[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ulo[d] = o[d] - 1;
        ucnt[d] = vd[d] + 2;
        if (kp.small_dim[d] && ucnt[d] > kp.nc[d]) { ulo[d] = 0; ucnt[d] = kp.nc[d]; }
    }
    const int32_t U = ucnt[0] * ucnt[1] * ucnt[2];
    int32_t myrank = INT_MAX, mystart = 0, mylen = 0, myoff = 0;
    if (lane < U) {
        const int32_t ux = lane % ucnt[0], uy = (lane / ucnt[0]) % ucnt[1], uz = lane / (ucnt[0] * ucnt[1]);
        const int32_t fx = ulo[0] + ux, fy = ulo[1] + uy, fz = ulo[2] + uz;   // block-frame cell
        myrank = rank_tab[lin_cell(kp, wrap_cell(fx, kp.nc[0]), wrap_cell(fy, kp.nc[1]), wrap_cell(fz, kp.nc[2]))];
        mystart = cell_start[myrank];
        mylen = cell_start[myrank + 1] - mystart;
        // cell offset from the block origin, packed as three signed bytes
        myoff = ((fx - o[0]) & 0xFF) | (((fy - o[1]) & 0xFF) << 8) | (((fz - o[2]) & 0xFF) << 16);
    }
    int32_t pos = 0;
    for (int m = 0; m < U; ++m) pos += (__builtin_amdgcn_readlane(myrank, m) < myrank) ? 1 : 0;
    pos = lane < U ? pos : lane;                                    // idle lanes keep their slot
    const int32_t s_start = __builtin_amdgcn_ds_permute(pos * 4, mystart);
    const int32_t s_len = __builtin_amdgcn_ds_permute(pos * 4, mylen);
    const int32_t s_off = __builtin_amdgcn_ds_permute(pos * 4, myoff);
    int32_t s_incl = s_len;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t t = __shfl_up(s_incl, d, kWave);
        if (lane >= d) s_incl += t;
    }
    const int32_t total = __builtin_amdgcn_readlane(s_incl, kWave - 1);

    const float4* __restrict__ xw = reinterpret_cast<const float4*>(x32);
    const float cl0 = kp.cell_len32[0], cl1 = kp.cell_len32[1], cl2 = kp.cell_len32[2];
    const bool wrap_any = kp.small_dim[0] | kp.small_dim[1] | kp.small_dim[2];

    for (int32_t ib = i_lo; ib < i_hi; ib += kWave) {            // i particles, 64 at a time
        const int32_t ie = (i_hi - ib) < kWave ? i_hi : ib + kWave;
        // lane li holds particle ib + li: in-cell offsets and its row count
        float wix = 0.f, wiy = 0.f, wiz = 0.f;
        int32_t run = 0;
        if (lane < ie - ib) {
            const float4 w = xw[ib + lane];
            wix = w.x; wiy = w.y; wiz = w.z;
            run = kDirect ? offset[ib + lane] : 0;
        }
        for (int32_t kb = 0; kb < total; kb += kWave) {           // candidates, 64 at a time
            const int32_t k = kb + lane;
            const bool valid = k < total;
            // sorted union cell holding candidate k: binary search on the prefix
            int32_t m = 0;
#pragma unroll
            for (int step = 32; step > 0; step >>= 1) {
                const int32_t probe = __shfl(s_incl, m + step - 1, kWave);
                m = (probe <= k) ? m + step : m;
            }
            m = m < kWave ? m : kWave - 1;
            const int32_t cs = __shfl(s_start, m, kWave);
            const int32_t cin = __shfl(s_incl, m, kWave);
            const int32_t cln = __shfl(s_len, m, kWave);
            const int32_t cof = __shfl(s_off, m, kWave);
            const int32_t j = valid ? cs + (k - (cin - cln)) : -1;
            const float4 wj = xw[valid ? j : 0];
            const float pjx = wj.x + (float)(int8_t)(cof & 0xFF) * cl0;
            const float pjy = wj.y + (float)(int8_t)((cof >> 8) & 0xFF) * cl1;
            const float pjz = wj.z + (float)(int8_t)((cof >> 16) & 0xFF) * cl2;
            // walk the block's cells in rank order; inside cell g the i
            // side sits at whole-cell offset delta_g from the block origin,
            // which is folded into the candidate positions once per cell
            int32_t g = -1, g_end = ib, code = -1;
            float qx = 0.f, qy = 0.f, qz = 0.f;
            for (int32_t i = ib; i < ie; ++i) {
                while (i >= g_end) {                               // next non-empty block cell
                    ++g;
                    do { ++code; } while (!((code & 1) < vd[0] && ((code >> 1) & 1) < vd[1] && (code >> 2) < vd[2]));
                    g_end = cell_start[r0 + g + 1];
                    qx = pjx - (float)(code & 1) * cl0;
                    qy = pjy - (float)((code >> 1) & 1) * cl1;
                    qz = pjz - (float)(code >> 2) * cl2;
                }
                const int li = i - ib;
                float dx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wix), li)) - qx;
                float dy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wiy), li)) - qy;
                float dz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wiz), li)) - qz;
                if (wrap_any) {
                    dx = kp.small_dim[0] ? min_image32(dx, kp.L32[0]) : dx;
                    dy = kp.small_dim[1] ? min_image32(dy, kp.L32[1]) : dy;
                    dz = kp.small_dim[2] ? min_image32(dz, kp.L32[2]) : dz;
                }
                const float r2 = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
                const bool cand = valid && j != i;
                bool hit = cand && r2 < kp.list_lo32;
                const bool amb = cand && !hit && r2 < kp.list_hi32;
                if (__ballot(amb)) {
                    if (amb) hit = exact_hit(kp, x, N, i, j);
                }
                const uint64_t mask = __ballot(hit);
                const int32_t base = __builtin_amdgcn_readlane(run, li);
                const int32_t at = base + lanes_below(mask);
                const int32_t cnt = (int32_t)__popcll(mask);
                if (kDirect) {
                    if (hit) index[at] = j;
                } else {
                    if (hit && at < slab_k) slab[(int64_t)i * slab_k + at] = j;
                    if (base + cnt > slab_k && lane == 0) atomicOr(flag, 1);
                }
                run = (lane == li) ? base + cnt : run;
            }
        }
        if (!kDirect && lane < ie - ib) offset[ib + lane] = run;
    }
}

// blk counts the 2x2x2 blocks of all systems of a batch in turn; kW waves
// per workgroup, one block per wave
template <bool kDirect, bool kB, int kW>
__global__ __launch_bounds__(kW * kWave) void k_nlist(KParams kp, BatchView bv, int32_t n_blocks, int32_t n,
                                                      const double* __restrict__ x, const float* __restrict__ x32,
                                                      const int32_t* __restrict__ cell_start,
                                                      const int32_t* __restrict__ rank_tab,
                                                      int32_t* __restrict__ offset, int32_t* __restrict__ index,
                                                      int64_t capacity, int32_t* __restrict__ slab, int32_t slab_k,
                                                      int32_t* __restrict__ flag, Gate gate)
{
    if (gated_off(gate)) return;
    const int32_t blk = xcd_logical_id(blockIdx.x, gridDim.x) * kW + threadIdx.x / kWave;
    if (blk >= n_blocks) return;
    if (kDirect && (*flag == 0 || (int64_t)offset[n] > capacity)) return;
    if constexpr (kB) {
        const int32_t sy = find_segment(bv.b_off, bv.n_sys, blk);
        nlist_block<kDirect>(bv.kps[sy], blk - bv.b_off[sy], n, x, x32, cell_start, rank_tab, offset, index, slab,
                             slab_k, flag);
    } else {
        nlist_block<kDirect>(kp, blk, n, x, x32, cell_start, rank_tab, offset, index, slab, slab_k, flag);
    }
}

// ---- lane-per-particle builder ----

constexpr SortNet kNet27 = make_sort_net(27);
static_assert(kNet27.count == 156, "27-key odd-even merge network");

template <bool kDirect>
__device__ __forceinline__ void nlist_lane(const KParams& kp, int32_t i, int32_t n, const double* __restrict__ x,
                                           const float* __restrict__ x32, const uint32_t* __restrict__ cell_xyz,
                                           const int32_t* __restrict__ cell_start,
                                           const int32_t* __restrict__ rank_tab, int32_t* __restrict__ offset,
                                           int32_t* __restrict__ index, int32_t* __restrict__ slab,
                                           int32_t slab_k, int32_t* __restrict__ flag)
{
    const int64_t N = n;
    const uint32_t me = cell_xyz[i];
    const int32_t cx = (int32_t)(me & 1023u), cy = (int32_t)((me >> 10) & 1023u), cz = (int32_t)(me >> 20);
    // stencil keys: rank << 5 | code, code = (dx+1) + 3 (dy+1) + 9 (dz+1)
    uint32_t key[27];
#pragma unroll
    for (int c = 0; c < 27; ++c) {
        const int dx = c % 3 - 1, dy = (c / 3) % 3 - 1, dz = c / 9 - 1;
        const int32_t r = rank_tab[lin_cell(kp, wrap_cell(cx + dx, kp.nc[0]), wrap_cell(cy + dy, kp.nc[1]),
                                            wrap_cell(cz + dz, kp.nc[2]))];
        key[c] = ((uint32_t)r << 5) | (uint32_t)c;
    }
#pragma unroll
    for (int c = 0; c < kNet27.count; ++c) {
        const uint32_t u = key[kNet27.a[c]], v = key[kNet27.b[c]];
        key[kNet27.a[c]] = u < v ? u : v;
        key[kNet27.b[c]] = u < v ? v : u;
    }
    const float4 wi = reinterpret_cast<const float4*>(x32)[i];
    const float4* __restrict__ xw = reinterpret_cast<const float4*>(x32);
    const float cl0 = kp.cell_len32[0], cl1 = kp.cell_len32[1], cl2 = kp.cell_len32[2];
    int32_t cnt = 0;
    int32_t* __restrict__ out = kDirect ? index + offset[i] : slab + (int64_t)i * slab_k;
    const int32_t cap = kDirect ? INT_MAX : slab_k;
    const bool coded = !kDirect && n <= kSlabJMask;
    // Loads run ahead of the tests: the next cell's bounds are requested when
    // a cell starts, candidates are tested two at a time while the two after
    // them are in flight, and a cell's first two are requested as the
    // previous cell ends.
    int32_t j0 = cell_start[key[0] >> 5], j1 = cell_start[(key[0] >> 5) + 1];
    float4 wa = xw[j0 < j1 ? j0 : i];
    float4 wb = xw[j0 + 1 < j1 ? j0 + 1 : i];
    auto test = [&](int32_t j, const float4& wj, float qx, float qy, float qz, uint32_t tagc) {
        const float dx = qx - wj.x, dy = qy - wj.y, dz = qz - wj.z;
        const float r2 = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
        bool hit = j != i && r2 < kp.list_lo32;
        if (j != i && !hit && r2 < kp.list_hi32) hit = exact_hit(kp, x, N, i, j);
        if (hit) {
            if (cnt < cap) out[cnt] = (int32_t)((uint32_t)j | tagc);
            ++cnt;
        }
    };
#pragma unroll
    for (int q = 0; q < 27; ++q) {
        int32_t j0n = 0, j1n = 0;
        if (q + 1 < 27) {
            const int32_t rn = (int32_t)(key[q + 1] >> 5);
            j0n = cell_start[rn];
            j1n = cell_start[rn + 1];
        }
        const int c = (int)(key[q] & 31u);
        const uint32_t tagc = coded ? ((uint32_t)(c % 3) | ((uint32_t)((c / 3) % 3) << 2) |
                                       ((uint32_t)(c / 9) << 4)) << kSlabCodeShift
                                    : 0u;
        // i's cell-relative position minus the cell's whole-cell offset
        const float qx = wi.x - (float)(c % 3 - 1) * cl0;
        const float qy = wi.y - (float)((c / 3) % 3 - 1) * cl1;
        const float qz = wi.z - (float)(c / 9 - 1) * cl2;
        for (int32_t j = j0; j < j1; j += 2) {
            const float4 w0 = wa, w1 = wb;
            const bool two = j + 1 < j1;
            // the pair after this one inside the cell (clamped to its last
            // candidate; the next cell's first two are requested below)
            const int32_t last = j1 - 1;
            wa = xw[j + 2 < last ? j + 2 : last];
            wb = xw[j + 3 < last ? j + 3 : last];
            test(j, w0, qx, qy, qz, tagc);
            if (two) test(j + 1, w1, qx, qy, qz, tagc);
        }
        wa = xw[j0n < j1n ? j0n : i];
        wb = xw[j0n + 1 < j1n ? j0n + 1 : i];
        j0 = j0n;
        j1 = j1n;
    }
    if (!kDirect) {
        offset[i] = cnt;
        if (cnt > slab_k) atomicOr(flag, 1);
    }
}

// workgroups of the direct pass (a few per compute unit)
constexpr int32_t kDirectGrid = 2048;

template <bool kDirect, bool kB, int kW>
__global__ __launch_bounds__(kW * kWave) void k_nlist_lanes(KParams kp, BatchView bv, int32_t n,
                                                            const double* __restrict__ x,
                                                            const float* __restrict__ x32,
                                                            const uint32_t* __restrict__ cell_xyz,
                                                            const int32_t* __restrict__ cell_start,
                                                            const int32_t* __restrict__ rank_tab,
                                                            int32_t* __restrict__ offset,
                                                            int32_t* __restrict__ index, int64_t capacity,
                                                            int32_t* __restrict__ slab, int32_t slab_k,
                                                            int32_t* __restrict__ flag, Gate gate)
{
    if (gated_off(gate)) return;
    if (kDirect && (*flag == 0 || (int64_t)offset[n] > capacity)) return;
    // (the direct pass runs on a capped grid, each lane taking every
    // gridDim-th group of rows: it is launched for every build and returns
    // at once unless the slab overflowed)
    const int32_t g0 = xcd_logical_id(blockIdx.x, gridDim.x);
    for (int64_t b = g0; b * (kW * kWave) < n; b += kDirect ? gridDim.x : (int64_t)n) {
        const int32_t i = (int32_t)(b * (kW * kWave)) + (int32_t)threadIdx.x;
        if (i >= n) return;
        if constexpr (kB)
            nlist_lane<kDirect>(bv.kps[bv.sys_of[i]], i, n, x, x32, cell_xyz, cell_start, rank_tab, offset, index,
                                slab, slab_k, flag);
        else
            nlist_lane<kDirect>(kp, i, n, x, x32, cell_xyz, cell_start, rank_tab, offset, index, slab, slab_k,
                                flag);
    }
}

template <bool kDirect, int kW>
void launch_nlist_lanes(const KParams& kp, const BatchView& bv, int32_t n, const double* x, const float* x32,
                        const uint32_t* cell_xyz, const int32_t* cell_start, const int32_t* rank_tab,
                        int32_t* offset, int32_t* index, int64_t capacity, int32_t* slab, int32_t slab_k,
                        int32_t* flag, hipStream_t s, Gate gate)
{
    const int32_t blocks = ceil_div(n, kW * kWave);
    const dim3 grid(kDirect && blocks > kDirectGrid ? kDirectGrid : blocks), block(kW * kWave);
    if (bv.kps)
        hipLaunchKernelGGL((k_nlist_lanes<kDirect, true, kW>), grid, block, 0, s, kp, bv, n, x, x32, cell_xyz,
                           cell_start, rank_tab, offset, index, capacity, slab, slab_k, flag, gate);
    else
        hipLaunchKernelGGL((k_nlist_lanes<kDirect, false, kW>), grid, block, 0, s, kp, bv, n, x, x32, cell_xyz,
                           cell_start, rank_tab, offset, index, capacity, slab, slab_k, flag, gate);
}

template <bool kDirect>
void launch_nlist_lanes(int waves, const KParams& kp, const BatchView& bv, int32_t n, const double* x,
                        const float* x32, const uint32_t* cell_xyz, const int32_t* cell_start,
                        const int32_t* rank_tab, int32_t* offset, int32_t* index, int64_t capacity,
                        int32_t* slab, int32_t slab_k, int32_t* flag, hipStream_t s, Gate gate)
{
    if (waves == 1)
        launch_nlist_lanes<kDirect, 1>(kp, bv, n, x, x32, cell_xyz, cell_start, rank_tab, offset, index, capacity,
                                       slab, slab_k, flag, s, gate);
    else if (waves == 2)
        launch_nlist_lanes<kDirect, 2>(kp, bv, n, x, x32, cell_xyz, cell_start, rank_tab, offset, index, capacity,
                                       slab, slab_k, flag, s, gate);
    else
        launch_nlist_lanes<kDirect, 4>(kp, bv, n, x, x32, cell_xyz, cell_start, rank_tab, offset, index, capacity,
                                       slab, slab_k, flag, s, gate);
}

template <bool kDirect, int kW>
void launch_nlist_pass(const KParams& kp, const BatchView& bv, int32_t n_blocks, int32_t n, const double* x,
                       const float* x32, const int32_t* cell_start, const int32_t* rank_tab, int32_t* offset,
                       int32_t* index, int64_t capacity, int32_t* slab, int32_t slab_k, int32_t* flag,
                       hipStream_t s, Gate gate)
{
    const dim3 grid(ceil_div(n_blocks, kW)), block(kW * kWave);
    if (bv.kps)
        hipLaunchKernelGGL((k_nlist<kDirect, true, kW>), grid, block, 0, s, kp, bv, n_blocks, n, x, x32, cell_start,
                           rank_tab, offset, index, capacity, slab, slab_k, flag, gate);
    else
        hipLaunchKernelGGL((k_nlist<kDirect, false, kW>), grid, block, 0, s, kp, bv, n_blocks, n, x, x32,
                           cell_start, rank_tab, offset, index, capacity, slab, slab_k, flag, gate);
}

template <bool kDirect>
void launch_nlist_pass(int waves, const KParams& kp, const BatchView& bv, int32_t n_blocks, int32_t n,
                       const double* x, const float* x32, const int32_t* cell_start, const int32_t* rank_tab,
                       int32_t* offset, int32_t* index, int64_t capacity, int32_t* slab, int32_t slab_k,
                       int32_t* flag, hipStream_t s, Gate gate)
{
    if (waves == 1)
        launch_nlist_pass<kDirect, 1>(kp, bv, n_blocks, n, x, x32, cell_start, rank_tab, offset, index, capacity,
                                      slab, slab_k, flag, s, gate);
    else if (waves == 2)
        launch_nlist_pass<kDirect, 2>(kp, bv, n_blocks, n, x, x32, cell_start, rank_tab, offset, index, capacity,
                                      slab, slab_k, flag, s, gate);
    else
        launch_nlist_pass<kDirect, 4>(kp, bv, n_blocks, n, x, x32, cell_start, rank_tab, offset, index, capacity,
                                      slab, slab_k, flag, s, gate);
}

// ---- tile builder ----
//
// One workgroup per tile of kTileX x kTileY x kTileZ cells (consecutive
// Morton ranks, so the tile's particles are one index range).  The union of
// its cells' stencils, (kTileX+2) x (kTileY+2) x (kTileZ+2) cells, is staged
// in LDS: each union cell's particles in index order, as FP32 positions in
// one tile frame (in-cell offset plus the cell's whole-cell offset from the
// frame origin) with the particle index.  Each tile cell's 27 stencil cells
// are put in ascending rank once, by one lane, with the same sorting
// network, and stored as LDS ranges.  Each lane then walks its particle's
// ranges in that order, one candidate per step, so its row comes out
// ascending; the walk is one flat loop over all of the particle's
// candidates, so lanes whose k-th stencil cells differ in size do not wait
// for each other cell by cell.  Candidates come from LDS, so the walk issues
// no global loads besides the row stores.  In a grid narrower than the
// union (fewer than 10 x 6 x 6 cells) a cell can appear in the union at two
// places, as two periodic images, and is staged twice; every tile cell's
// 27 stencil cells are still distinct cells (3 or more per side), each at
// the image next to it, so no candidate is seen twice.  Tiles whose
// neighbourhood overflows the LDS take the lane builder's walk over global
// memory.

constexpr int kTUX = kTileX + 2, kTUY = kTileY + 2, kTUZ = kTileZ + 2;
constexpr int kTU = kTUX * kTUY * kTUZ;          // union cells of a tile
constexpr int kTC = kTileX * kTileY * kTileZ;     // cells of a tile
// staged particles per tile: the workgroup's lanes (sized to the tile
// population's mean + 1.5 sigma) times 2.9, a little above the union's
// 360 / 128 cells per tile cell.  At density 3 (7 waves, 1,312 slots) the
// union's ~1,100 particles fluctuate by ~33, and the LDS use (39 KB) lets
// four workgroups share a compute unit.
template <int kW>
constexpr int tile_pos() { return (kW * kWave * 29 / 10 + 15) / 16 * 16; }
// union cell whose origin is the tile frame's origin (keeps |positions| small)
constexpr int kTFX = kTileX / 2 + 1, kTFY = kTileY / 2 + 1, kTFZ = kTileZ / 2 + 1;
// candidates a lane tests per step of the walk, and their operands
constexpr int kStepW = 2;
// a byte offset past the slab rows of every tile (a tile's rows span less
// than INT32_MAX - 4 tile_pos bytes, or it is left to the lane builder)
constexpr int32_t kDropOff = 0x7FFFFFF0;
struct StepW {
    float4 w[kStepW];
};
// stencil entry: LDS start | LDS end << 12 | slab code << kSlabCodeShift
// (the code is 0 when the slab is not coded), so an entry's code bits are
// the ones a slab entry carries
static_assert(tile_pos<16>() < 4096, "12-bit LDS offsets in the stencil entries");
static_assert(kTC * 27 * 4 >= tile_pos<16>() * 2, "the staging map fits in the stencil table");

// exclusive prefix of v over the workgroup (kW waves); total gets the sum
template <int kW>
__device__ __forceinline__ int32_t tile_excl_scan(int32_t v, int32_t* s_w, int32_t& total)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int32_t incl = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int32_t t = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += t;
    }
    if (lane == kWave - 1) s_w[w] = incl;
    __syncthreads();
    int32_t base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kW; ++k) {
        const int32_t sw = s_w[k];
        base += k < w ? sw : 0;
        tot += sw;
    }
    total = tot;
    return base + incl - v;
}

// The tile's system and cells: tile origin o (cells), its extent v (clipped
// at the high faces) and its particle range [i_lo, i_hi).
struct TileGeom {
    const KParams* P;
    int32_t o0, o1, o2, v0, v1, v2;
    int32_t i_lo, i_hi;
};

template <bool kB>
__device__ __forceinline__ TileGeom tile_geom(const KParams& kp, const BatchView& bv, int32_t tile,
                                              const int32_t* __restrict__ cell_start,
                                              const int32_t* __restrict__ rank_tab)
{
    TileGeom g;
    int32_t t_loc = tile;
    g.P = &kp;
    if constexpr (kB) {
        const int32_t sy = find_segment(bv.t_off, bv.n_sys, tile);
        g.P = &bv.kps[sy];
        t_loc = tile - bv.t_off[sy];
    }
    const KParams& P = *g.P;
    const int32_t tx = t_loc % P.nt[0], ty = (t_loc / P.nt[0]) % P.nt[1], tz = t_loc / (P.nt[0] * P.nt[1]);
    g.o0 = tx * kTileX; g.o1 = ty * kTileY; g.o2 = tz * kTileZ;
    g.v0 = min(kTileX, P.nc[0] - g.o0); g.v1 = min(kTileY, P.nc[1] - g.o1); g.v2 = min(kTileZ, P.nc[2] - g.o2);
    // the origin cell has the tile's smallest rank; its cells are the next v0 v1 v2 ranks
    const int32_t r0 = rank_tab[lin_cell(P, g.o0, g.o1, g.o2)];
    g.i_lo = cell_start[r0];
    g.i_hi = cell_start[r0 + g.v0 * g.v1 * g.v2];
    return g;
}

template <bool kB, int kW>
__global__ __launch_bounds__(kW * kWave) void k_nlist_tiles(KParams kp, BatchView bv, int32_t n_tiles, int32_t n,
                                                            const double* __restrict__ x,
                                                            const float* __restrict__ x32,
                                                            const uint32_t* __restrict__ cell_xyz,
                                                            const int32_t* __restrict__ cell_start,
                                                            const int32_t* __restrict__ rank_tab,
                                                            int32_t* __restrict__ offset,
                                                            int32_t* __restrict__ slab, int32_t slab_k,
                                                            int32_t* __restrict__ flag,
                                                            int32_t* __restrict__ rest, Gate gate)
{
    if (gated_off(gate)) return;
    constexpr int kThreads = kW * kWave;
    static_assert(kThreads >= kTU && kThreads >= kTC, "one thread per union cell and per tile cell");
    __shared__ int32_t s_rank[kTU];
    __shared__ int32_t s_gstart[kTU];
    __shared__ int32_t s_lstart[kTU + 1];
    constexpr int kTilePos = tile_pos<kW>();
    __shared__ float4 s_pos[kTilePos + kStepW - 1];   // spare slots: a step's reads may run past the end
    // (two spare entries: the walk reads up to two entries past a cell's last)
    __shared__ uint32_t s_sten[kTC * 27 + 2];  // before the sort: union cell of every staged slot
    __shared__ uint8_t s_nne[kTC];
    __shared__ int32_t s_w[kW];
    uint16_t* s_seg = reinterpret_cast<uint16_t*>(s_sten);

    const int32_t tile = xcd_logical_id(blockIdx.x, gridDim.x);
    if (tile >= n_tiles) return;
    const TileGeom g = tile_geom<kB>(kp, bv, tile, cell_start, rank_tab);
    if (g.i_lo == g.i_hi) return;
    const KParams& P = *g.P;
    const int tid = threadIdx.x;
    // (the tile's slab rows are addressed with 32-bit byte offsets)
    const bool fits = (int64_t)(g.i_hi - g.i_lo) * slab_k * 4 + 4 * kTilePos < INT32_MAX;

    // ---- union cells: thread u owns union cell u ----
    int32_t cnt = 0;
    if (fits && tid < kTU) {
        const int32_t ux = tid % kTUX, uy = (tid / kTUX) % kTUY, uz = tid / (kTUX * kTUY);
        int32_t rank = INT_MAX, gs = 0;
        if (ux < g.v0 + 2 && uy < g.v1 + 2 && uz < g.v2 + 2) {
            rank = rank_tab[lin_cell(P, wrap_cell(g.o0 + ux - 1, P.nc[0]), wrap_cell(g.o1 + uy - 1, P.nc[1]),
                                     wrap_cell(g.o2 + uz - 1, P.nc[2]))];
            gs = cell_start[rank];
            cnt = cell_start[rank + 1] - gs;
        }
        s_rank[tid] = rank;
        s_gstart[tid] = gs;
    }
    int32_t total;
    const int32_t ls = tile_excl_scan<kW>(cnt, s_w, total);
    if (!fits || total > kTilePos) {
        // left to the lane builder's walk over global memory (k_nlist_tile_rest)
        if (tid == 0) rest[1 + atomicAdd(rest, 1)] = tile;
        return;
    }
    if (tid < kTU) {
        s_lstart[tid] = ls;
        for (int32_t k = 0; k < cnt; ++k) s_seg[ls + k] = (uint16_t)tid;
    }
    if (tid == 0) s_lstart[kTU] = total;
    __syncthreads();

    // ---- staging: every union particle in the tile frame ----
    const float4* __restrict__ xw = reinterpret_cast<const float4*>(x32);
    const float cl0 = P.cell_len32[0], cl1 = P.cell_len32[1], cl2 = P.cell_len32[2];
    for (int32_t p = tid; p < total; p += kThreads) {
        const int32_t u = s_seg[p];
        const int32_t j = s_gstart[u] + (p - s_lstart[u]);
        const float4 w = xw[j];
        const int32_t ux = u % kTUX, uy = (u / kTUX) % kTUY, uz = u / (kTUX * kTUY);
        s_pos[p] = make_float4(w.x + (float)(ux - kTFX) * cl0, w.y + (float)(uy - kTFY) * cl1,
                               w.z + (float)(uz - kTFZ) * cl2, __int_as_float(j));
    }
    __syncthreads();

    // ---- each tile cell's non-empty stencil cells in ascending rank ----
    if (tid < kTC) {
        const int32_t lx = tid % kTileX, ly = (tid / kTileX) % kTileY, lz = tid / (kTileX * kTileY);
        if (lx < g.v0 && ly < g.v1 && lz < g.v2) {
            uint32_t key[27];
#pragma unroll
            for (int c = 0; c < 27; ++c) {
                const int32_t u = (lx + c % 3) + kTUX * ((ly + (c / 3) % 3) + kTUY * (lz + c / 9));
                key[c] = ((uint32_t)s_rank[u] << 5) | (uint32_t)c;
            }
#pragma unroll
            for (int c = 0; c < kNet27.count; ++c) {
                const uint32_t a = key[kNet27.a[c]], b = key[kNet27.b[c]];
                key[kNet27.a[c]] = a < b ? a : b;
                key[kNet27.b[c]] = a < b ? b : a;
            }
            uint32_t* st = s_sten + tid * 27;
            const uint32_t cmask = n <= kSlabJMask ? ~0u : 0u;     // uncoded slab: no code bits
            int32_t m = 0;
#pragma unroll
            for (int q = 0; q < 27; ++q) {
                const int32_t c = (int32_t)(key[q] & 31u);
                const int32_t ex = c % 3, ey = (c / 3) % 3, ez = c / 9;
                const int32_t u = (lx + ex) + kTUX * ((ly + ey) + kTUY * (lz + ez));
                const uint32_t code = ((uint32_t)ex | ((uint32_t)ey << 2) | ((uint32_t)ez << 4)) & cmask;
                const int32_t a = s_lstart[u], b = s_lstart[u + 1];
                if (a < b) st[m++] = (uint32_t)a | ((uint32_t)b << 12) | (code << kSlabCodeShift);
            }
            s_nne[tid] = (uint8_t)m;
            // the walk reads up to two entries past a cell's last: empty
            // ranges at slot 0
            for (int32_t q = m; q < 27; ++q) st[q] = 0u;
        } else {
            for (int32_t q = 0; q < 27; ++q) s_sten[tid * 27 + q] = 0u;
        }
    }
    if (tid < 2) s_sten[kTC * 27 + tid] = 0u;
    __syncthreads();

    // ---- the walk: one lane per particle of the tile ----
    // kStepW candidates of a cell per step (slots k, k + 1, ...; slots past
    // the cell's end idle, and their reads may be the spare slots past the
    // staged range, never used).  The next step's candidates and the stencil
    // entry after the next are requested from LDS before the current ones
    // are tested; two steps per loop turn alternate the buffers.
    const float lo = P.tile_lo32, hi = P.tile_hi32;
    const int64_t N = n;
    constexpr uint32_t kCodeBits = ~0u << kSlabCodeShift;
    // The tile's slab rows through a buffer resource: a row longer than the
    // slab width runs on into the next rows of the tile (stores past the
    // tile's last row are dropped by the range check); such a row sets the
    // flag, and the whole slab is then discarded for the direct pass.
    const int32_t n_here = g.i_hi - g.i_lo;
    const auto rows = __builtin_amdgcn_make_buffer_rsrc(slab + (int64_t)g.i_lo * slab_k, (short)0,
                                                        n_here * slab_k * (int32_t)sizeof(int32_t), 0x00020000);
    for (int32_t i = g.i_lo + tid; i < g.i_hi; i += kThreads) {
        const uint32_t me = cell_xyz[i];
        const int32_t lx = (int32_t)(me & 1023u) - g.o0, ly = (int32_t)((me >> 10) & 1023u) - g.o1,
                      lz = (int32_t)(me >> 20) - g.o2;
        const int32_t ui = (lx + 1) + kTUX * ((ly + 1) + kTUY * (lz + 1));
        const float4 wi = s_pos[s_lstart[ui] + (i - s_gstart[ui])];
        const int32_t ci = lx + kTileX * (ly + kTileY * lz);
        const uint32_t* st = s_sten + ci * 27;
        const int32_t nne = s_nne[ci];                   // >= 1: i's own cell is in its stencil
        // byte offset of this lane's next entry in the tile's slab rows
        const int32_t row0 = (i - g.i_lo) * slab_k * (int32_t)sizeof(int32_t);
        int32_t rb = row0;
        // walk state: the current stencil entry cur (its cell's slots end at
        // bits 12..23, its slab code in the top bits), the candidate slot k,
        // and the entry after cur (ent_n, at index pn)
        uint32_t cur = st[0];
        int32_t pn = 1;
        uint32_t ent_n = st[1];
        int32_t k = (int32_t)(cur & 0xFFFu);
        // the FP32 test of one candidate: hit (inside lo) or band (between
        // lo and hi, to be decided by the FP64 rule)
        auto pre = [&](const float4& w, bool valid, bool& band) {
            const float dx = wi.x - w.x, dy = wi.y - w.y, dz = wi.z - w.z;
            const float r2 = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
            const bool near = r2 < lo;
            band = valid && !near && r2 < hi;
            // i itself has r2 = 0 < lo, so the band never holds it
            return valid && near && __float_as_int(w.w) != i;
        };
        auto store = [&](const float4& w, uint32_t ent, bool hit) {
            // every lane stores: a miss at an offset past the rows' range,
            // which the buffer's range check drops (no branch per candidate)
            __builtin_amdgcn_raw_buffer_store_b32((int32_t)((ent & kCodeBits) | (uint32_t)__float_as_int(w.w)),
                                                  rows, hit ? rb : kDropOff, 0, 0);
            rb += hit ? (int32_t)sizeof(int32_t) : 0;
        };
        // one step on the candidates at slots k .. k + kStepW - 1 (those below
        // the cell's end), advancing the state and requesting the next step's
        // candidates into nxt and the entry after the next; false when the
        // walk has ended.  Past the end the state runs on into the following
        // entries of the table (the next cell's, or the zeroed ones), whose
        // slots are valid reads and never tested.
        auto step = [&](const StepW& cw, StepW& nxt) {
            const uint32_t ent = cur;
            const int32_t left = (int32_t)((ent >> 12) & 0xFFFu) - k;   // >= 1
            const bool adv = left <= kStepW;
            k = adv ? (int32_t)(ent_n & 0xFFFu) : k + kStepW;
            cur = adv ? ent_n : cur;
            pn += adv ? 1 : 0;
            const float4* p = s_pos + k;
#pragma unroll
            for (int m = 0; m < kStepW; ++m) nxt.w[m] = p[m];
            ent_n = st[pn];
            bool hit[kStepW], band[kStepW];
            bool any_band = false;
#pragma unroll
            for (int m = 0; m < kStepW; ++m) {
                hit[m] = pre(cw.w[m], m == 0 || m < left, band[m]);
                any_band = any_band || band[m];
            }
            // the band is rare: the wave branches once per step on its ballot
            if (__builtin_expect(__ballot(any_band) != 0ull, 0)) {
#pragma unroll
                for (int m = 0; m < kStepW; ++m)
                    if (band[m]) hit[m] = exact_hit(P, x, N, i, __float_as_int(cw.w[m].w));
            }
#pragma unroll
            for (int m = 0; m < kStepW; ++m) store(cw.w[m], ent, hit[m]);
            return pn <= nne;
        };
        StepW s0, s1;
#pragma unroll
        for (int m = 0; m < kStepW; ++m) s0.w[m] = s_pos[k + m];
        for (;;) {
            if (!step(s0, s1)) break;
            if (!step(s1, s0)) break;
        }
        const int32_t row = (rb - row0) / (int32_t)sizeof(int32_t);
        offset[i] = row;
        if (row > slab_k) atomicOr(flag, 1);
    }
}

// Tiles the tile builder left (neighbourhood over the LDS capacity):
// rest[0] tiles listed in rest[1..], their particles walked by the lane
// builder.
template <bool kB>
__global__ __launch_bounds__(kBlock) void k_nlist_tile_rest(KParams kp, BatchView bv, int32_t n,
                                                            const double* __restrict__ x,
                                                            const float* __restrict__ x32,
                                                            const uint32_t* __restrict__ cell_xyz,
                                                            const int32_t* __restrict__ cell_start,
                                                            const int32_t* __restrict__ rank_tab,
                                                            int32_t* __restrict__ offset,
                                                            int32_t* __restrict__ slab, int32_t slab_k,
                                                            int32_t* __restrict__ flag,
                                                            const int32_t* __restrict__ rest, Gate gate)
{
    if (gated_off(gate)) return;
    const int32_t count = rest[0];
    for (int32_t t = blockIdx.x; t < count; t += gridDim.x) {
        const TileGeom g = tile_geom<kB>(kp, bv, rest[1 + t], cell_start, rank_tab);
        for (int32_t i = g.i_lo + (int32_t)threadIdx.x; i < g.i_hi; i += kBlock)
            nlist_lane<false>(*g.P, i, n, x, x32, cell_xyz, cell_start, rank_tab, offset, nullptr, slab, slab_k,
                              flag);
    }
}

template <bool kB, int kW>
void launch_nlist_tiles_t(const KParams& kp, const BatchView& bv, int32_t n_tiles, int32_t n, const double* x,
                          const float* x32, const uint32_t* cell_xyz, const int32_t* cell_start,
                          const int32_t* rank_tab, int32_t* offset, int32_t* slab, int32_t slab_k, int32_t* flag,
                          int32_t* rest, hipStream_t s, Gate gate)
{
    hipLaunchKernelGGL((k_nlist_tiles<kB, kW>), dim3(n_tiles), dim3(kW * kWave), 0, s, kp, bv, n_tiles, n, x, x32,
                       cell_xyz, cell_start, rank_tab, offset, slab, slab_k, flag, rest, gate);
}

// tile pass, then the pass over the tiles it left; rest[0] must be 0
template <bool kB>
void launch_nlist_tiles(int waves, const KParams& kp, const BatchView& bv, int32_t n_tiles, int32_t n,
                        const double* x, const float* x32, const uint32_t* cell_xyz, const int32_t* cell_start,
                        const int32_t* rank_tab, int32_t* offset, int32_t* slab, int32_t slab_k, int32_t* flag,
                        int32_t* rest, hipStream_t s, Gate gate)
{
#define DPD_TILE_CASE(W)                                                                                         \
    launch_nlist_tiles_t<kB, W>(kp, bv, n_tiles, n, x, x32, cell_xyz, cell_start, rank_tab, offset, slab, slab_k, \
                                flag, rest, s, gate)
    if (waves <= 6) DPD_TILE_CASE(6);
    else if (waves <= 7) DPD_TILE_CASE(7);
    else if (waves <= 8) DPD_TILE_CASE(8);
    else if (waves <= 10) DPD_TILE_CASE(10);
    else if (waves <= 12) DPD_TILE_CASE(12);
    else DPD_TILE_CASE(16);
#undef DPD_TILE_CASE
    const int grid = n_tiles < 1024 ? n_tiles : 1024;
    hipLaunchKernelGGL((k_nlist_tile_rest<kB>), dim3(grid), dim3(kBlock), 0, s, kp, bv, n, x, x32, cell_xyz,
                       cell_start, rank_tab, offset, slab, slab_k, flag, (const int32_t*)rest, gate);
}

}  // namespace

// Waves per tile workgroup: the mean particle count of a tile plus 1.5
// standard deviations (a tile with more particles walks the rest in a
// second round), at least enough threads for one per union cell.
int nlist_tile_waves(int32_t n, int32_t n_cells)
{
    const double mean = (double)kTC * (double)n / (double)(n_cells > 0 ? n_cells : 1);
    const double need = mean + 1.5 * std::sqrt(mean);
    int w = (int)std::ceil(need / kWave);
    constexpr int kMinW = (kTU + kWave - 1) / kWave;
    return w < kMinW ? kMinW : (w > 16 ? 16 : w);
}

namespace {

// CSR list from the slab: one wave per 64 consecutive rows writes their
// entries [offset[i0], offset[i0 + 64]) in order, one entry per lane.
__global__ __launch_bounds__(kBlock) void k_nlist_compact(int32_t n, const int32_t* __restrict__ offset,
                                                          int64_t capacity, const int32_t* __restrict__ slab,
                                                          int32_t slab_k, const int32_t* __restrict__ flag,
                                                          int32_t* __restrict__ index)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t i0 = ((int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave) * kWave;
    const int32_t mask = n <= kSlabJMask ? kSlabJMask : -1;      // strips coded stencil offsets
    if (i0 >= n || *flag != 0 || (int64_t)offset[n] > capacity) return;
    const int32_t ni = n - i0 < kWave ? (int32_t)(n - i0) : kWave;
    const int32_t own = (int32_t)i0 + (lane < ni ? lane : ni - 1);
    const int32_t e0 = offset[i0], e1 = offset[i0 + ni];
    int32_t rend = offset[own + 1];
    const int32_t prev = __shfl_up(rend, 1, kWave);
    int32_t rstart = lane == 0 ? e0 : prev;
    if (lane >= ni) { rstart = e1; rend = e1; }
    for (int32_t eb = e0; eb < e1; eb += kWave) {
        // rows ra..rb-1 overlap this batch; walk their ends with readlane
        const int32_t e = eb + lane;
        const int32_t ra = (int32_t)__popcll(__ballot(lane < ni && rend <= eb));
        const int32_t rb = (int32_t)__popcll(__ballot(lane < ni && rstart < eb + kWave));
        int32_t r = ra;
        int32_t rs = __builtin_amdgcn_readlane(rstart, ra < kWave ? ra : kWave - 1);
        for (int32_t q = ra; q < rb; ++q) {
            const int32_t t = __builtin_amdgcn_readlane(rend, q);
            if (e >= t) { r = q + 1; rs = t; }
        }
        if (e < e1) index[e] = slab[(i0 + r) * slab_k + (e - rs)] & mask;
    }
}

__global__ void k_nlist_check(int32_t n, const int32_t* __restrict__ offset, int64_t capacity,
                              int32_t* __restrict__ status, Gate gate)
{
    if (gated_off(gate)) return;
    if (threadIdx.x == 0 && blockIdx.x == 0 && (int64_t)offset[n] > capacity)
        atomicOr(status, 1 /* DPD_STATUS_NLIST_OVERFLOW */);
}

}  // namespace

// Slots per row of the scratch slab: about 2.5 times the mean neighbour
// count plus a margin (rows that do not fit fall back to the direct pass).
int32_t nlist_slab_width(double density, double rl2)
{
    const double mean = 4.18879020478639 * density * rl2 * sqrt(rl2);
    int32_t k = (int32_t)(2.5 * mean + 24.0);
    k = k < 48 ? 48 : k;
    return (k + 15) / 16 * 16;
}

// The tile and lane builders pack a rank and a 5-bit stencil code into 32
// bits; beyond 2^27 cells the block builder takes over.
static bool ranks_fit(const uint32_t* cell_xyz, int32_t n_cells)
{
    return cell_xyz && n_cells < (1 << 27);
}

bool nlist_slab_coded(int kind, const uint32_t* cell_xyz, int32_t n_cells, int32_t n)
{
    return (kind == 0 || kind == 2) && ranks_fit(cell_xyz, n_cells) && n <= kSlabJMask;
}

hipError_t launch_nlist(const KParams& kp, const BatchView& bv, int32_t n_cells, int32_t n_blocks, int32_t n_tiles,
                        int32_t n, const double* x, const float* x32, const uint32_t* cell_xyz,
                        const int32_t* cell_start, const int32_t* rank_tab, int32_t* offset, int32_t* index,
                        int64_t capacity, int32_t* slab, int32_t slab_k, int32_t* flag, int32_t* tile_rest,
                        int32_t* status, int32_t* scan_part, int waves, int kind, bool compact, hipStream_t s,
                        Gate gate)
{
    if (n <= 0) return hipSuccess;
    hipError_t e;
    const bool tiles = kind == 0 && ranks_fit(cell_xyz, n_cells);
    const bool lanes = tiles || (kind == 2 && ranks_fit(cell_xyz, n_cells));
    if ((e = launch_zero3(offset + n, flag, tiles ? tile_rest : nullptr, s, gate)) != hipSuccess) return e;
    if (tiles) {
        const int tw = nlist_tile_waves(n, n_cells);
        if (bv.kps)
            launch_nlist_tiles<true>(tw, kp, bv, n_tiles, n, x, x32, cell_xyz, cell_start, rank_tab, offset, slab,
                                     slab_k, flag, tile_rest, s, gate);
        else
            launch_nlist_tiles<false>(tw, kp, bv, n_tiles, n, x, x32, cell_xyz, cell_start, rank_tab, offset, slab,
                                      slab_k, flag, tile_rest, s, gate);
    } else if (lanes)
        launch_nlist_lanes<false>(waves, kp, bv, n, x, x32, cell_xyz, cell_start, rank_tab, offset, index, capacity,
                                  slab, slab_k, flag, s, gate);
    else
        launch_nlist_pass<false>(waves, kp, bv, n_blocks, n, x, x32, cell_start, rank_tab, offset, index, capacity,
                                 slab, slab_k, flag, s, gate);
    if ((e = launch_scan(offset, (int64_t)n + 1, scan_part, s, gate)) != hipSuccess) return e;
    if (status) {
        hipLaunchKernelGGL(k_nlist_check, dim3(1), dim3(64), 0, s, n, (const int32_t*)offset, capacity, status, gate);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // without compaction the CSR index is left unwritten unless a row
    // overflowed the slab (then the direct pass below writes it).  The
    // compaction takes no gate: after a step that kept the last build's
    // rows it copies those rows again.
    if (compact)
        hipLaunchKernelGGL(k_nlist_compact, dim3(ceil_div(ceil_div(n, kWave), kWavesPerBlock)), dim3(kBlock), 0,
                           s, n, (const int32_t*)offset, capacity, (const int32_t*)slab, slab_k,
                           (const int32_t*)flag, index);
    // rows that overflowed the slab: the lane builder's walk writes the CSR
    // rows directly (the same rows the tile builder would give)
    if (lanes)
        launch_nlist_lanes<true>(waves, kp, bv, n, x, x32, cell_xyz, cell_start, rank_tab, offset, index, capacity,
                                 slab, slab_k, flag, s, gate);
    else
        launch_nlist_pass<true>(waves, kp, bv, n_blocks, n, x, x32, cell_start, rank_tab, offset, index, capacity,
                                slab, slab_k, flag, s, gate);
    return hipGetLastError();
}

hipError_t launch_nlist_compact(int32_t n, const int32_t* offset, int64_t capacity, const int32_t* slab,
                                int32_t slab_k, const int32_t* flag, int32_t* index, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nlist_compact, dim3(ceil_div(ceil_div(n, kWave), kWavesPerBlock)), dim3(kBlock), 0, s, n,
                       offset, capacity, slab, slab_k, flag, index);
    return hipGetLastError();
}

hipError_t launch_nlist_check(int32_t n, const int32_t* offset, int64_t capacity, int32_t* status,
                              hipStream_t s)
{
    if (!status) return hipSuccess;
    hipLaunchKernelGGL(k_nlist_check, dim3(1), dim3(64), 0, s, n, offset, capacity, status, nullptr);
    return hipGetLastError();
}

}  // namespace dpd
