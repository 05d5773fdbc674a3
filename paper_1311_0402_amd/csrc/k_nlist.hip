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
// A count pass sizes the rows, a scan makes the CSR offsets, a fill pass
// writes them.
#include <climits>

#include "dpd_launch.h"

namespace dpd {

namespace {

constexpr int kWavesPerBlock = kBlock / kWave;

__device__ __forceinline__ int32_t wrap_cell(int32_t c, int32_t n)
{
    c = c < 0 ? c + n : c;
    return c >= n ? c - n : c;
}

__device__ __forceinline__ int32_t lin_cell(const KParams& kp, int32_t cx, int32_t cy, int32_t cz)
{
    return cx + kp.nc[0] * (cy + kp.nc[1] * cz);
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

template <bool kFill>
__global__ __launch_bounds__(kBlock) void k_nlist(KParams kp, int32_t n, const double* __restrict__ x,
                                                  const float* __restrict__ x32,
                                                  const uint32_t* __restrict__ cell_xyz,
                                                  const int32_t* __restrict__ cell_start,
                                                  const int32_t* __restrict__ rank_tab,
                                                  int32_t* __restrict__ offset, int32_t* __restrict__ index,
                                                  int64_t capacity)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t blk = xcd_logical_id(blockIdx.x, gridDim.x) * kWavesPerBlock + threadIdx.x / kWave;
    if (blk >= kp.n_blocks) return;
    if (kFill && (int64_t)offset[n] > capacity) return;   // overflow flagged by the check kernel
    const int64_t N = n;

    // ---- the block and its particle range ----
    int32_t bx, by, bz;
    morton_unrank(blk, kp.nb[0], kp.nb[1], kp.nb[2], kp.nbits_b, &bx, &by, &bz);
    const int32_t o[3] = {2 * bx, 2 * by, 2 * bz};                 // block origin (cells)
    int32_t nv = 1;
#pragma unroll
    for (int d = 0; d < 3; ++d) nv *= (kp.nc[d] - o[d] >= 2) ? 2 : 1;
    const int32_t r0 = rank_tab[lin_cell(kp, o[0], o[1], o[2])];
    const int32_t i_lo = cell_start[r0], i_hi = cell_start[r0 + nv];
    if (i_lo == i_hi) return;

    // ---- union of the block's stencils: lane m < U owns union cell m ----
    int32_t ulo[3], ucnt[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int32_t v = (kp.nc[d] - o[d] >= 2) ? 2 : 1;
        ulo[d] = o[d] - 1;
        ucnt[d] = v + 2;
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

    const float cl0 = kp.cell_len32[0], cl1 = kp.cell_len32[1], cl2 = kp.cell_len32[2];
    const bool wrap_any = kp.small_dim[0] | kp.small_dim[1] | kp.small_dim[2];

    for (int32_t ib = i_lo; ib < i_hi; ib += kWave) {            // i particles, 64 at a time
        const int32_t ni = (i_hi - ib) < kWave ? (i_hi - ib) : kWave;
        // lane li holds particle ib + li in the block frame
        float pix = 0.f, piy = 0.f, piz = 0.f;
        int32_t run = 0;
        if (lane < ni) {
            const int32_t i = ib + lane;
            const uint32_t c = cell_xyz[i];
            pix = x32[i] + (float)((int32_t)(c & 1023u) - o[0]) * cl0;
            piy = x32[N + i] + (float)((int32_t)((c >> 10) & 1023u) - o[1]) * cl1;
            piz = x32[2 * N + i] + (float)((int32_t)(c >> 20) - o[2]) * cl2;
            if (kFill) run = offset[i];
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
            const int32_t j = valid ? cs + (k - (cin - cln)) : 0;
            const float ox = (float)(int8_t)(cof & 0xFF), oy = (float)(int8_t)((cof >> 8) & 0xFF),
                        oz = (float)(int8_t)((cof >> 16) & 0xFF);
            const float pjx = x32[j] + ox * cl0;
            const float pjy = x32[N + j] + oy * cl1;
            const float pjz = x32[2 * N + j] + oz * cl2;
            for (int32_t li = 0; li < ni; ++li) {
                const int32_t i = ib + li;
                float dx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pix), li)) - pjx;
                float dy = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(piy), li)) - pjy;
                float dz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(piz), li)) - pjz;
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
                if (kFill) {
                    const int32_t base = __builtin_amdgcn_readlane(run, li);
                    if (hit) index[base + lanes_below(mask)] = j;
                }
                run = (lane == li) ? run + (int32_t)__popcll(mask) : run;
            }
        }
        if (!kFill && lane < ni) offset[ib + lane] = run;
    }
}

__global__ void k_nlist_check(int32_t n, const int32_t* __restrict__ offset, int64_t capacity,
                              int32_t* __restrict__ status)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && (int64_t)offset[n] > capacity)
        atomicOr(status, 1 /* DPD_STATUS_NLIST_OVERFLOW */);
}

int nlist_groups(const KParams& kp) { return ceil_div(kp.n_blocks, kWavesPerBlock); }

}  // namespace

hipError_t launch_nlist_count(const KParams& kp, int32_t n, const double* x, const float* x32,
                              const uint32_t* cell_xyz, const int32_t* cell_start, const int32_t* rank_tab,
                              int32_t* offset, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nlist<false>, dim3(nlist_groups(kp)), dim3(kBlock), 0, s, kp, n, x, x32, cell_xyz,
                       cell_start, rank_tab, offset, (int32_t*)nullptr, (int64_t)0);
    return hipGetLastError();
}

hipError_t launch_nlist_check(int32_t n, const int32_t* offset, int64_t capacity, int32_t* status,
                              hipStream_t s)
{
    if (!status) return hipSuccess;
    hipLaunchKernelGGL(k_nlist_check, dim3(1), dim3(64), 0, s, n, offset, capacity, status);
    return hipGetLastError();
}

hipError_t launch_nlist_fill(const KParams& kp, int32_t n, const double* x, const float* x32,
                             const uint32_t* cell_xyz, const int32_t* cell_start, const int32_t* rank_tab,
                             const int32_t* offset, int32_t* index, int64_t capacity, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nlist<true>, dim3(nlist_groups(kp)), dim3(kBlock), 0, s, kp, n, x, x32, cell_xyz,
                       cell_start, rank_tab, const_cast<int32_t*>(offset), index, capacity);
    return hipGetLastError();
}

}  // namespace dpd
