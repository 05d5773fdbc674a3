// k_border.hip -- border determination and ghost packing for a spatial
// decomposition (Sec. 3.6 and Algorithm 6 of the paper): flag the particles
// within `width` of each face of the brick, a multi-block scan of the
// flags' per-block counts (one segment per face), compaction into ascending
// send lists, and packing / unpacking of the ghost records.
//
// Flags: 6 bits per particle (bit f = 2 d + s set when the particle is
// within `width` of face f: s = 0 the low face, x_d < lo_d + width; s = 1
// the high face, x_d >= hi_d - width), for the faces the caller selects.
// Counts: cnt[f * n_blk + b] = flagged particles of face f in block b of
// kBlock particles.  One exclusive scan over the 6 n_blk counts (faces one
// after another) gives every (face, block) its first slot in the
// concatenated send lists, whose face offsets are the scan at f * n_blk.
// Compaction: a particle's slot is its block's slot plus the flagged
// particles before it in the block (wave ballots and the waves' counts),
// so each list ascends.
#include "dpd_launch.h"

namespace dpd {

namespace {

constexpr int kFaces = 6;
constexpr int kWaves = kBlock / kWave;

struct BorderBox {
    double lo_w[3];      // lo + width: the low face's band is x < lo_w
    double hi_w[3];      // hi - width: the high face's band is x >= hi_w
};

__device__ __forceinline__ uint32_t face_bits(const BorderBox& bb, int32_t mask, const double* __restrict__ x,
                                              int64_t N, int32_t i)
{
    uint32_t m = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double xd = x[d * N + i];
        m |= (xd < bb.lo_w[d] ? 1u : 0u) << (2 * d);
        m |= (xd >= bb.hi_w[d] ? 1u : 0u) << (2 * d + 1);
    }
    return m & (uint32_t)mask;
}

// flags and per-block counts (block b covers particles [b kBlock, (b + 1) kBlock))
__global__ __launch_bounds__(kBlock) void k_border_flag(BorderBox bb, int32_t face_mask, int32_t n,
                                                        const double* __restrict__ x, uint8_t* __restrict__ flags,
                                                        int32_t* __restrict__ cnt, int32_t n_blk)
{
    __shared__ int32_t s_c[kFaces][kWaves];
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t m = i < n ? face_bits(bb, face_mask, x, n, i) : 0u;
    if (i < n) flags[i] = (uint8_t)m;
#pragma unroll
    for (int f = 0; f < kFaces; ++f) {
        const int32_t c = (int32_t)__popcll(__ballot((m >> f) & 1u));
        if (lane == 0) s_c[f][w] = c;
    }
    __syncthreads();
    if (threadIdx.x < kFaces) {
        int32_t t = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) t += s_c[threadIdx.x][q];
        cnt[threadIdx.x * (int64_t)n_blk + blockIdx.x] = t;
    }
}

// send lists from the scanned counts (slot[f n_blk + b] = first slot of face
// f in block b; slot[6 n_blk] = total); block 0 also writes the face offsets
__global__ __launch_bounds__(kBlock) void k_border_compact(int32_t n, const uint8_t* __restrict__ flags,
                                                           const int32_t* __restrict__ slot, int32_t n_blk,
                                                           int32_t* __restrict__ send_offset,
                                                           int32_t* __restrict__ send_index, int64_t capacity,
                                                           int32_t* __restrict__ status)
{
    __shared__ int32_t s_c[kFaces][kWaves];
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t total = slot[kFaces * (int64_t)n_blk];
    if (blockIdx.x == 0 && threadIdx.x <= kFaces) {
        send_offset[threadIdx.x] = threadIdx.x < kFaces ? slot[threadIdx.x * (int64_t)n_blk] : (int32_t)total;
        if (threadIdx.x == 0 && total > capacity && status) atomicOr(status, 8 /* DPD_STATUS_HALO_OVERFLOW */);
    }
    const uint32_t m = i < n ? flags[i] : 0u;
    uint64_t bal[kFaces];
#pragma unroll
    for (int f = 0; f < kFaces; ++f) {
        bal[f] = __ballot((m >> f) & 1u);
        if (lane == 0) s_c[f][w] = (int32_t)__popcll(bal[f]);
    }
    __syncthreads();
    if (total > capacity) return;
#pragma unroll
    for (int f = 0; f < kFaces; ++f) {
        if (!((m >> f) & 1u)) continue;
        int32_t before = 0;
        for (int q = 0; q < w; ++q) before += s_c[f][q];
        const int64_t at = (int64_t)slot[f * (int64_t)n_blk + blockIdx.x] + before + lanes_below(bal[f]);
        send_index[at] = i;
    }
}

struct Shift {
    double s[kFaces][3];
};

// face of concatenated record r (the number of face offsets 1..6 at or below r)
__device__ __forceinline__ int face_of(const int32_t* __restrict__ off, int32_t r)
{
    int f = 0;
#pragma unroll
    for (int q = 1; q < kFaces; ++q) f += off[q] <= r ? 1 : 0;
    return f;
}

__global__ __launch_bounds__(kBlock) void k_border_pack(int32_t n, const double* __restrict__ x,
                                                        const double* __restrict__ v,
                                                        const uint32_t* __restrict__ tag,
                                                        const uint8_t* __restrict__ type,
                                                        const int32_t* __restrict__ send_offset,
                                                        const int32_t* __restrict__ send_index, int64_t capacity,
                                                        Shift sh, dpd_ghost* __restrict__ out,
                                                        int32_t* __restrict__ status)
{
    const int64_t total = send_offset[kFaces];
    if (total > capacity) return;
    const int64_t N = n;
    for (int32_t r = blockIdx.x * kBlock + threadIdx.x; r < total; r += gridDim.x * kBlock) {
        const int f = face_of(send_offset, r);
        const int32_t j = send_index[r];
        if (j < 0 || j >= n) {                  // not a list of this state
            if (status) atomicOr(status, 8 /* DPD_STATUS_HALO_OVERFLOW */);
            continue;
        }
        dpd_ghost g;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            g.x[d] = x[d * N + j] + sh.s[f][d];
            g.v[d] = v[d * N + j];
        }
        g.tag = tag[j];
        g.type = (uint32_t)type[j];
        out[r] = g;
    }
}

__global__ __launch_bounds__(kBlock) void k_border_unpack(const dpd_ghost* __restrict__ in,
                                                          const int32_t* __restrict__ d_count, int64_t capacity,
                                                          int32_t n_dst, int32_t first, double* __restrict__ x,
                                                          double* __restrict__ v, uint32_t* __restrict__ tag,
                                                          uint8_t* __restrict__ type, int32_t* __restrict__ status)
{
    const int64_t count = *d_count;
    if (count > capacity || (int64_t)first + count > n_dst) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && status) atomicOr(status, 8 /* DPD_STATUS_HALO_OVERFLOW */);
        return;
    }
    const int64_t N = n_dst;
    for (int32_t r = blockIdx.x * kBlock + threadIdx.x; r < count; r += gridDim.x * kBlock) {
        const dpd_ghost g = in[r];
        const int64_t i = (int64_t)first + r;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            x[d * N + i] = g.x[d];
            v[d * N + i] = g.v[d];
        }
        tag[i] = g.tag;
        type[i] = (uint8_t)g.type;
    }
}

constexpr int kMaxStrideBlocks = 2048;   // grid of the grid-stride pack / unpack

}  // namespace

BorderWs border_ws_layout(int32_t n)
{
    BorderWs w;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = (o + bytes + 255) & ~(size_t)255; return at; };
    const int32_t n_blk = ceil_div(n > 0 ? n : 1, kBlock);
    const int64_t items = (int64_t)kFaces * n_blk + 1;
    w.n_blk = n_blk;
    w.flags = take((size_t)(n > 0 ? n : 1));
    w.cnt = take((size_t)items * sizeof(int32_t));
    w.scan_part = take((size_t)ceil_div(items, kScanTile) * sizeof(int32_t) + 64);
    w.total = o;
    return w;
}

hipError_t launch_border_lists(int32_t n, const double* x, const double lo[3], const double hi[3], double width,
                               int32_t face_mask, int32_t* send_offset, int32_t* send_index, int64_t capacity,
                               int32_t* status, void* ws, hipStream_t s)
{
    const BorderWs L = border_ws_layout(n);
    uint8_t* flags = reinterpret_cast<uint8_t*>(static_cast<char*>(ws) + L.flags);
    int32_t* cnt = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + L.cnt);
    int32_t* part = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + L.scan_part);
    BorderBox bb;
    for (int d = 0; d < 3; ++d) {
        bb.lo_w[d] = lo[d] + width;
        bb.hi_w[d] = hi[d] - width;
    }
    const int64_t items = (int64_t)kFaces * L.n_blk + 1;
    hipError_t e;
    // every block writes its six counts; the last entry (the total after the
    // scan) starts at zero
    if ((e = launch_fill_i32(cnt + items - 1, 1, 0, s)) != hipSuccess) return e;
    if (n > 0)
        hipLaunchKernelGGL(k_border_flag, dim3(L.n_blk), dim3(kBlock), 0, s, bb, face_mask, n, x, flags, cnt,
                           L.n_blk);
    else if ((e = launch_fill_i32(cnt, items - 1, 0, s)) != hipSuccess)
        return e;
    if ((e = launch_scan(cnt, items, part, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_border_compact, dim3(L.n_blk), dim3(kBlock), 0, s, n, (const uint8_t*)flags,
                       (const int32_t*)cnt, L.n_blk, send_offset, send_index, capacity, status);
    return hipGetLastError();
}

hipError_t launch_border_pack(int32_t n, const double* x, const double* v, const uint32_t* tag, const uint8_t* type,
                              const int32_t* send_offset, const int32_t* send_index, int64_t capacity,
                              const double shift[18], dpd_ghost* out, int32_t* status, hipStream_t s)
{
    Shift sh;
    for (int f = 0; f < kFaces; ++f)
        for (int d = 0; d < 3; ++d) sh.s[f][d] = shift[3 * f + d];
    const int64_t want = (capacity + kBlock - 1) / kBlock;
    const int grid = (int)(want < 1 ? 1 : (want > kMaxStrideBlocks ? kMaxStrideBlocks : want));
    hipLaunchKernelGGL(k_border_pack, dim3(grid), dim3(kBlock), 0, s, n, x, v, tag, type, send_offset, send_index,
                       capacity, sh, out, status);
    return hipGetLastError();
}

hipError_t launch_border_unpack(const dpd_ghost* in, const int32_t* d_count, int64_t capacity, int32_t n_dst,
                                int32_t first, double* x, double* v, uint32_t* tag, uint8_t* type, int32_t* status,
                                hipStream_t s)
{
    const int64_t want = (capacity + kBlock - 1) / kBlock;
    const int grid = (int)(want < 1 ? 1 : (want > kMaxStrideBlocks ? kMaxStrideBlocks : want));
    hipLaunchKernelGGL(k_border_unpack, dim3(grid), dim3(kBlock), 0, s, in, d_count, capacity, n_dst, first, x, v,
                       tag, type, status);
    return hipGetLastError();
}

}  // namespace dpd
