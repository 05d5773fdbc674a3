// k_nlist.hip -- ordered neighbour list (Sec. 3.3 of the paper).
//
// One 64-lane wavefront owns one cell.  Its 27 surrounding cells (periodic)
// are put in ascending Morton rank, so their particle ranges, which the
// reordering made contiguous, concatenate into one strictly ascending
// candidate sequence (the paper's sorted stencil).  Lanes walk the
// candidates 64 at a time; for every particle i of the cell the wave
// ballots the distance test, and a lane's insertion point is the row's
// running count plus the number of hits in lower lanes (mbcnt).  Rows are
// therefore ascending and deterministic without atomics.  A count pass
// sizes the rows, a scan makes the CSR offsets, a fill pass writes them.
//
// The stencil lives in registers: lane m < 27 computes neighbour cell m, and
// the sorted order is read back with v_readlane, so no LDS and no barrier
// is needed and each wave may leave as soon as its cell is done.
#include <climits>

#include "dpd_launch.h"

namespace dpd {

namespace {

constexpr int kWavesPerBlock = kBlock / kWave;

struct Stencil {
    // per lane m < 27: first particle and exclusive/inclusive candidate
    // prefix of the m-th cell in ascending rank
    int32_t start, excl, incl;
    int32_t total;
};

__device__ __forceinline__ int32_t wrap_cell(int32_t c, int32_t n)
{
    c = c < 0 ? c + n : c;
    return c >= n ? c - n : c;
}

__device__ __forceinline__ Stencil make_stencil(const KParams& kp, const int32_t* __restrict__ cell_start,
                                                uint32_t packed)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t cx = (int32_t)(packed & 1023u);
    const int32_t cy = (int32_t)((packed >> 10) & 1023u);
    const int32_t cz = (int32_t)(packed >> 20);
    int32_t myrank = INT_MAX, mystart = 0, mylen = 0;
    if (lane < 27) {
        const int32_t nx = wrap_cell(cx + lane % 3 - 1, kp.nc[0]);
        const int32_t ny = wrap_cell(cy + (lane / 3) % 3 - 1, kp.nc[1]);
        const int32_t nz = wrap_cell(cz + lane / 9 - 1, kp.nc[2]);
        myrank = morton_rank(nx, ny, nz, kp.nc[0], kp.nc[1], kp.nc[2], kp.nbits);
        mystart = cell_start[myrank];
        mylen = cell_start[myrank + 1] - mystart;
    }
    // position of this lane's cell in ascending rank (ranks are distinct for n_c >= 3)
    int32_t pos = 0;
#pragma unroll
    for (int m = 0; m < 27; ++m) pos += (__builtin_amdgcn_readlane(myrank, m) < myrank) ? 1 : 0;
    // lane k takes the cell at sorted position k
    int32_t sstart = 0, slen = 0;
#pragma unroll
    for (int m = 0; m < 27; ++m) {
        const int32_t pm = __builtin_amdgcn_readlane(pos, m);
        const int32_t st = __builtin_amdgcn_readlane(mystart, m);
        const int32_t ln = __builtin_amdgcn_readlane(mylen, m);
        if (pm == lane) { sstart = st; slen = ln; }
    }
    int32_t incl = slen;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
        const int32_t t = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += t;
    }
    Stencil s;
    s.start = sstart;
    s.excl = incl - slen;
    s.incl = incl;
    s.total = __builtin_amdgcn_readlane(incl, 26);
    return s;
}

// candidate number k (0 <= k < total) -> particle index
__device__ __forceinline__ int32_t candidate(const Stencil& s, int32_t k)
{
    int32_t j = -1;
#pragma unroll
    for (int m = 0; m < 27; ++m) {
        const int32_t ex = __builtin_amdgcn_readlane(s.excl, m);
        const int32_t in = __builtin_amdgcn_readlane(s.incl, m);
        const int32_t st = __builtin_amdgcn_readlane(s.start, m);
        j = (k >= ex && k < in) ? st + (k - ex) : j;
    }
    return j;
}

template <bool kFill>
__global__ __launch_bounds__(kBlock) void k_nlist(KParams kp, int32_t n, const double* __restrict__ x,
                                                  const int32_t* __restrict__ cell_start,
                                                  const uint32_t* __restrict__ cell_xyz,
                                                  int32_t* __restrict__ offset, int32_t* __restrict__ index,
                                                  int64_t capacity)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t cell = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    if (cell >= kp.n_cells) return;
    const int32_t lo = cell_start[cell], hi = cell_start[cell + 1];
    if (lo == hi) return;
    if (kFill && (int64_t)offset[n] > capacity) return;   // overflow flagged by the check kernel

    const int64_t N = n;
    const Stencil st = make_stencil(kp, cell_start, cell_xyz[lo]);
    const double rl2 = kp.rl2;

    for (int32_t ib = lo; ib < hi; ib += kWave) {           // i particles, 64 at a time
        const int32_t ie = ib + kWave < hi ? ib + kWave : hi;
        int32_t run = 0;                                      // lane (i - ib) owns row i
        if (kFill && ib + lane < ie) run = offset[ib + lane];
        for (int32_t kb = 0; kb < st.total; kb += kWave) {   // candidates, 64 at a time
            const int32_t k = kb + lane;
            const bool valid = k < st.total;
            const int32_t j = valid ? candidate(st, k) : 0;
            const double xj = x[j], yj = x[N + j], zj = x[2 * N + j];
            for (int32_t i = ib; i < ie; ++i) {
                const double dx = min_image(x[i] - xj, kp.L[0], kp.halfL[0]);
                const double dy = min_image(x[N + i] - yj, kp.L[1], kp.halfL[1]);
                const double dz = min_image(x[2 * N + i] - zj, kp.L[2], kp.halfL[2]);
                const bool hit = valid && j != i && dist2(dx, dy, dz) < rl2;
                const uint64_t mask = __ballot(hit);
                const int li = i - ib;
                if (kFill) {
                    const int32_t base = __shfl(run, li, kWave);
                    if (hit) index[base + lanes_below(mask)] = j;
                }
                if (lane == li) run += __popcll(mask);
            }
        }
        if (!kFill && ib + lane < ie) offset[ib + lane] = run;
    }
}

__global__ void k_nlist_check(int32_t n, const int32_t* __restrict__ offset, int64_t capacity,
                              int32_t* __restrict__ status)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && (int64_t)offset[n] > capacity)
        atomicOr(status, 1 /* DPD_STATUS_NLIST_OVERFLOW */);
}

}  // namespace

hipError_t launch_nlist_count(const KParams& kp, int32_t n, const double* x, const int32_t* cell_start,
                              const uint32_t* cell_xyz, int32_t* offset, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nlist<false>, dim3(ceil_div(kp.n_cells, kWavesPerBlock)), dim3(kBlock), 0, s,
                       kp, n, x, cell_start, cell_xyz, offset, (int32_t*)nullptr, (int64_t)0);
    return hipGetLastError();
}

hipError_t launch_nlist_check(int32_t n, const int32_t* offset, int64_t capacity, int32_t* status,
                              hipStream_t s)
{
    if (!status) return hipSuccess;
    hipLaunchKernelGGL(k_nlist_check, dim3(1), dim3(64), 0, s, n, offset, capacity, status);
    return hipGetLastError();
}

hipError_t launch_nlist_fill(const KParams& kp, int32_t n, const double* x, const int32_t* cell_start,
                             const uint32_t* cell_xyz, const int32_t* offset, int32_t* index,
                             int64_t capacity, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nlist<true>, dim3(ceil_div(kp.n_cells, kWavesPerBlock)), dim3(kBlock), 0, s,
                       kp, n, x, cell_start, cell_xyz, const_cast<int32_t*>(offset), index, capacity);
    return hipGetLastError();
}

}  // namespace dpd
