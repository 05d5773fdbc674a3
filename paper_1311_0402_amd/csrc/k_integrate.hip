// k_integrate.hip -- velocity-Verlet phases (Eq (1) and Algorithm 1 of the
// paper, in the Groot-Warren form with velocity prediction lambda) and the
// per-step statistics ("calculate statistics" of Algorithm 1), all FP64.
//
// Phase 1 (k_vv1):  v_h = fma(dt/2, F, v);  x' = fma(dt, v_h, x) wrapped
//                   into [0, L) (add L if negative, then subtract L if >= L);
//                   v~ = fma(lambda dt, F, v) unless lambda = 1/2 (v~ = v_h).
// Phase 2 (k_vv2):  v = fma(dt/2, F_new, v_h), plus per-block partial sums
//                   of momentum and |v|^2 over a fixed grid; optionally
//                   followed by the next step's phase 1 on the same data
//                   (then v itself is not stored: the reorder takes v_h).
// k_reduce_final adds all partials in one fixed order (deterministic) and
// advances the device step counter.
#include "dpd_launch.h"

namespace dpd {

namespace {

// kp supplies the step sizes (shared by a batch's systems), L the box edge
// of particle i's system
__device__ __forceinline__ void vv1_one(const KParams& kp, double L, int32_t n, int32_t i, int k,
                                        const double* __restrict__ x, const double* __restrict__ v,
                                        const double* __restrict__ f, const uint32_t* __restrict__ tag,
                                        const uint8_t* __restrict__ type, double* __restrict__ bx,
                                        double* __restrict__ bv, double* __restrict__ bvt,
                                        uint32_t* __restrict__ btag, uint8_t* __restrict__ btype)
{
    const int64_t a = (int64_t)k * n + i;
    const double vh = __fma_rn(kp.half_dt, f[a], v[a]);
    double xn = __fma_rn(kp.dt, vh, x[a]);
    if (xn < 0.0) xn = xn + L;
    if (xn >= L) xn = xn - L;
    bx[a] = xn;
    bv[a] = vh;
    if (bvt) bvt[a] = __fma_rn(kp.lam_dt, f[a], v[a]);
    if (k == 0) {
        btag[i] = tag[i];
        btype[i] = type[i];
    }
}

template <bool kB>
__global__ __launch_bounds__(kBlock) void k_vv1(KParams kp, BatchView bat, int32_t n, const double* __restrict__ x,
                                                const double* __restrict__ v, const double* __restrict__ f,
                                                const uint32_t* __restrict__ tag,
                                                const uint8_t* __restrict__ type, double* __restrict__ bx,
                                                double* __restrict__ bv, double* __restrict__ bvt,
                                                uint32_t* __restrict__ btag, uint8_t* __restrict__ btype)
{
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    const int k = blockIdx.y;                       // component
    if (i >= n) return;
    if constexpr (kB)
        vv1_one(kp, bat.kps[bat.sys_of[i]].L[k], n, i, k, x, v, f, tag, type, bx, bv, bvt, btag, btype);
    else
        vv1_one(kp, kp.L[k], n, i, k, x, v, f, tag, type, bx, bv, bvt, btag, btype);
}

// Per-system statistics of a batch, in two fixed-order passes.  First one
// wave per 64-particle chunk (chunks are numbered system by system) sums
// momentum, |v|^2, potential energy and pairs over its particles into
// part[c][0..5]; then one block per system adds its chunks' sums and forms
// k_B T.  The totals go to row (*d_step - *base) of red (row 0 when base is
// null).
// With f given, the chunk pass first applies the step's second half-kick
// v = fma(dt/2, F, v) (the same arithmetic as k_vv2) and stores v.
__global__ __launch_bounds__(kBlock) void k_sys_chunks(BatchView bat, int32_t n, double* __restrict__ v,
                                                       const double* __restrict__ f, double half_dt,
                                                       const double* __restrict__ pe,
                                                       const int32_t* __restrict__ npair,
                                                       double* __restrict__ part)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t c = blockIdx.x * (kBlock / kWave) + (int32_t)(threadIdx.x / kWave);
    if (c >= bat.n_chunks) return;
    const int32_t sy = find_segment(bat.ch_off, bat.n_sys, c);
    const int32_t i = bat.p_off[sy] + (c - bat.ch_off[sy]) * kWave + lane;
    const int64_t N = n;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < bat.p_off[sy + 1]) {
        double vx = v[i], vy = v[N + i], vz = v[2 * N + i];
        if (f) {
            vx = __fma_rn(half_dt, f[i], vx);
            vy = __fma_rn(half_dt, f[N + i], vy);
            vz = __fma_rn(half_dt, f[2 * N + i], vz);
            v[i] = vx; v[N + i] = vy; v[2 * N + i] = vz;
        }
        acc[0] = vx; acc[1] = vy; acc[2] = vz;
        acc[3] = vx * vx + vy * vy + vz * vz;
        acc[4] = pe[i];
        acc[5] = (double)npair[i];
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1)
#pragma unroll
        for (int q = 0; q < 6; ++q) acc[q] += __shfl_down(acc[q], d, kWave);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 6; ++q) part[6 * (int64_t)c + q] = acc[q];
}

__global__ __launch_bounds__(kBlock) void k_sys_reduce(BatchView bat, const double* __restrict__ part,
                                                       double* __restrict__ red, const uint64_t* d_step,
                                                       const uint64_t* base, int32_t* status)
{
    __shared__ double s[6][kBlock];
    const int32_t sy = blockIdx.x;
    const int32_t lo = bat.p_off[sy], hi = bat.p_off[sy + 1];
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int32_t c = bat.ch_off[sy] + threadIdx.x; c < bat.ch_off[sy + 1]; c += kBlock)
#pragma unroll
        for (int q = 0; q < 6; ++q) acc[q] += part[6 * (int64_t)c + q];
    for (int q = 0; q < 6; ++q) s[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int wdt = kBlock / 2; wdt > 0; wdt >>= 1) {
        if (threadIdx.x < wdt)
            for (int q = 0; q < 6; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + wdt];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double nn = (double)(hi - lo);
        const double P0 = s[0][0], P1 = s[1][0], P2 = s[2][0], v2 = s[3][0];
        const double kbt = nn > 1.0 ? (v2 - (P0 * P0 + P1 * P1 + P2 * P2) / nn) / (3.0 * (nn - 1.0)) : 0.0;
        if (red) {
            const int64_t row = base ? (int64_t)(*d_step - *base) : 0;
            double* r = red + 8 * (row * bat.n_sys + sy);
            // (a batch rebuilds its lists every step)
            r[0] = P0; r[1] = P1; r[2] = P2; r[3] = v2; r[4] = s[4][0]; r[5] = 0.5 * s[5][0]; r[6] = kbt; r[7] = 1.0;
        }
        const double chk = P0 + P1 + P2 + v2 + s[4][0];
        if (status && !(chk - chk == 0.0)) atomicOr(status, 2 /* DPD_STATUS_NONFINITE */);
    }
}

// one thread: *dst = *src (a step counter snapshot) or *dst += 1 (src null)
__global__ void k_counter(uint64_t* dst, const uint64_t* src)
{
    if (threadIdx.x == 0) *dst = src ? *src : *dst + 1ull;
}

__global__ __launch_bounds__(kBlock) void k_sys_map(BatchView bat, int32_t n, uint16_t* __restrict__ sys_of)
{
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) sys_of[i] = (uint16_t)find_segment(bat.p_off, bat.n_sys, i);
}

__global__ __launch_bounds__(kBlock) void k_vv2(KParams kp, int32_t n, double* __restrict__ v,
                                                const double* __restrict__ f, double* __restrict__ part,
                                                const double* __restrict__ fred, int32_t n_fred,
                                                double* __restrict__ fsum, DriftArgs dr)
{
    __shared__ double s_p[kBlock / kWave], s_q[kBlock / kWave];
    const int k = blockIdx.y;
    const int64_t base = (int64_t)k * n;
    const double L = kp.L[k];
    double p = 0.0, q = 0.0;
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += kRedBlocks * kBlock) {
        double vn = v[base + i];
        if (f) vn = __fma_rn(kp.half_dt, f[base + i], vn);
        if (dr.bx) {
            // the next step's phase 1, as k_vv1 computes it from v = vn
            const double vh = __fma_rn(kp.half_dt, f[base + i], vn);
            double xn = __fma_rn(kp.dt, vh, dr.x[base + i]);
            if (xn < 0.0) xn = xn + L;
            if (xn >= L) xn = xn - L;
            dr.bx[base + i] = xn;
            dr.bv[base + i] = vh;
            if (dr.bvt) dr.bvt[base + i] = __fma_rn(kp.lam_dt, f[base + i], vn);
            if (k == 0) {
                dr.btag[i] = dr.tag[i];
                dr.btype[i] = dr.type[i];
            }
        } else if (f) {
            v[base + i] = vn;
        }
        p += vn;
        q += vn * vn;
    }
    if (k == 0 && fred) {
        // fold the force kernel's per-block (PE, pairs) partials, strided by
        // this block, so the final sum has only kRedBlocks terms per column
        __shared__ double s_fa[kBlock], s_fb[kBlock];
        double fa = 0.0, fb = 0.0;
        for (int32_t m = blockIdx.x + kRedBlocks * threadIdx.x; m < n_fred; m += kRedBlocks * kBlock) {
            fa += fred[2 * (int64_t)m];
            fb += fred[2 * (int64_t)m + 1];
        }
        s_fa[threadIdx.x] = fa;
        s_fb[threadIdx.x] = fb;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                s_fa[threadIdx.x] += s_fa[threadIdx.x + w];
                s_fb[threadIdx.x] += s_fb[threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            fsum[2 * blockIdx.x] = s_fa[0];
            fsum[2 * blockIdx.x + 1] = s_fb[0];
        }
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        p += __shfl_down(p, d, kWave);
        q += __shfl_down(q, d, kWave);
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) { s_p[w] = p; s_q[w] = q; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tp = 0.0, tq = 0.0;
        for (int m = 0; m < kBlock / kWave; ++m) { tp += s_p[m]; tq += s_q[m]; }
        part[2 * ((int64_t)k * kRedBlocks + blockIdx.x)] = tp;
        part[2 * ((int64_t)k * kRedBlocks + blockIdx.x) + 1] = tq;
    }
}

// The first phase of a step with a Verlet skin, in place on the sorted state
// (the same arithmetic as k_vv2 followed by k_vv1), one thread per particle
// over a fixed grid of kRedBlocks blocks so the momentum and |v|^2 partials
// keep k_vv2's layout.  Besides the new x and v~ it writes the packed copies
// the list-free steps' force pass reads, and raises the rebuild flag when a
// particle is more than skin / 2 from where the last rebuild saw it.
__global__ __launch_bounds__(kBlock) void k_drift_skin(KParams kp, int32_t n, SkinDriftArgs d,
                                                       double* __restrict__ part, const double* __restrict__ fred,
                                                       int32_t n_fred, double* __restrict__ fsum)
{
    __shared__ double s_p[3][kBlock / kWave], s_q[3][kBlock / kWave];
    const int64_t N = n;
    double p[3] = {0.0, 0.0, 0.0}, q[3] = {0.0, 0.0, 0.0};
    bool far = false;
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += kRedBlocks * kBlock) {
        const uint32_t cc = d.cell_xyz[i];
        const int32_t cell[3] = {(int32_t)(cc & 1023u), (int32_t)((cc >> 10) & 1023u), (int32_t)(cc >> 20)};
        double xn[3], vh[3], vt[3], r2 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int64_t a = k * N + i;
            const double fk = d.f[a];
            const double vn = __fma_rn(kp.half_dt, fk, d.v[a]);     // phase 2 of the previous step
            vh[k] = __fma_rn(kp.half_dt, fk, vn);                   // phase 1 of this step
            double x = __fma_rn(kp.dt, vh[k], d.x[a]);
            if (x < 0.0) x = x + kp.L[k];
            if (x >= kp.L[k]) x = x - kp.L[k];
            xn[k] = x;
            vt[k] = d.vt ? __fma_rn(kp.lam_dt, fk, vn) : vh[k];
            d.x[a] = x;
            d.v[a] = vh[k];
            if (d.vt) d.vt[a] = vt[k];
            p[k] += vn;
            q[k] += vn * vn;
            const double dk = min_image(x - d.xref[a], kp.L[k], kp.halfL[k]);
            r2 = __fma_rn(dk, dk, r2);
        }
        far = far || r2 > d.disp2;
        if (d.x32) {
            // offset from the cell the particle had at the last rebuild,
            // taken to the periodic image next to that cell
            float o[3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                o[k] = (float)min_image(xn[k] - (double)cell[k] * kp.cell_len[k], kp.L[k], kp.halfL[k]);
            reinterpret_cast<float4*>(d.x32)[i] = make_float4(o[0], o[1], o[2], __uint_as_float(d.tag[i]));
        }
        if (d.v32)
            reinterpret_cast<float4*>(d.v32)[i] =
                make_float4((float)vt[0], (float)vt[1], (float)vt[2], __uint_as_float((uint32_t)d.type[i]));
        if (d.x64) {
            double4 px, pv;
            px.x = xn[0]; px.y = xn[1]; px.z = xn[2]; px.w = __longlong_as_double((long long)d.tag[i]);
            pv.x = vt[0]; pv.y = vt[1]; pv.z = vt[2]; pv.w = __longlong_as_double((long long)d.type[i]);
            reinterpret_cast<double4*>(d.x64)[i] = px;
            reinterpret_cast<double4*>(d.v64)[i] = pv;
        }
    }
    if (__ballot(far) && lane_id() == 0) atomicOr(d.flag, 1);
    if (fred) {
        // the force kernel's (PE, pairs) partials folded as k_vv2 does
        __shared__ double s_fa[kBlock], s_fb[kBlock];
        double fa = 0.0, fb = 0.0;
        for (int32_t m = blockIdx.x + kRedBlocks * threadIdx.x; m < n_fred; m += kRedBlocks * kBlock) {
            fa += fred[2 * (int64_t)m];
            fb += fred[2 * (int64_t)m + 1];
        }
        s_fa[threadIdx.x] = fa;
        s_fb[threadIdx.x] = fb;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                s_fa[threadIdx.x] += s_fa[threadIdx.x + w];
                s_fb[threadIdx.x] += s_fb[threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            fsum[2 * blockIdx.x] = s_fa[0];
            fsum[2 * blockIdx.x + 1] = s_fb[0];
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int dd = kWave / 2; dd > 0; dd >>= 1) {
            p[k] += __shfl_down(p[k], dd, kWave);
            q[k] += __shfl_down(q[k], dd, kWave);
        }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 3; ++k) { s_p[k][w] = p[k]; s_q[k][w] = q[k]; }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int k = threadIdx.x;
        double tp = 0.0, tq = 0.0;
        for (int m = 0; m < kBlock / kWave; ++m) { tp += s_p[k][m]; tq += s_q[k][m]; }
        part[2 * ((int64_t)k * kRedBlocks + blockIdx.x)] = tp;
        part[2 * ((int64_t)k * kRedBlocks + blockIdx.x) + 1] = tq;
    }
}

// the step's statistics from the per-workgroup partials, in a fixed order
__global__ __launch_bounds__(kBlock) void k_reduce_final(int32_t n, const double* __restrict__ red_part,
                                                         int n_red, int red_stride,
                                                         const double* __restrict__ fred_part,
                                                         int n_fred, double* __restrict__ red,
                                                         double* __restrict__ stats, uint64_t* d_step,
                                                         int32_t* status, const int32_t* __restrict__ rebuilt)
{
    // eight columns (the momentum and |v|^2 partials of the three components,
    // the force pass's PE and pair partials): each thread sums its strided
    // share of every column in ascending order, then one tree per column
    // (the same order as one column at a time, with one pass of loads)
    __shared__ double s[8][kBlock];
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (red_part) {
        for (int m = threadIdx.x; m < n_red; m += kBlock) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                acc[2 * k] += red_part[2 * ((int64_t)k * red_stride + m)];
                acc[2 * k + 1] += red_part[2 * ((int64_t)k * red_stride + m) + 1];
            }
        }
    }
    if (fred_part) {
        for (int m = threadIdx.x; m < n_fred; m += kBlock) {
            acc[6] += fred_part[2 * (int64_t)m];
            acc[7] += fred_part[2 * (int64_t)m + 1];
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) s[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int c = 0; c < 8; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + w];
        }
        __syncthreads();
    }
    double P[3] = {s[0][0], s[2][0], s[4][0]};
    double v2 = 0.0;
    v2 += s[1][0];
    v2 += s[3][0];
    v2 += s[5][0];
    const double pe = s[6][0], pairs = s[7][0];
    if (threadIdx.x == 0) {
        const double nn = (double)n;
        const double kbt = n > 1 ? (v2 - (P[0] * P[0] + P[1] * P[1] + P[2] * P[2]) / nn) / (3.0 * (nn - 1.0)) : 0.0;
        if (red) {
            red[0] = P[0]; red[1] = P[1]; red[2] = P[2];
            red[3] = v2; red[4] = pe; red[5] = pairs; red[6] = kbt;
            red[7] = rebuilt ? (*rebuilt != 0 ? 1.0 : 0.0) : 1.0;
        }
        if (stats) { stats[0] = pe; stats[1] = pairs; }
        const double chk = P[0] + P[1] + P[2] + v2 + pe;
        if (status && !(chk - chk == 0.0)) atomicOr(status, 2 /* DPD_STATUS_NONFINITE */);
        if (d_step) *d_step = *d_step + 1ull;
    }
}

}  // namespace

hipError_t launch_vv1(const KParams& kp, const BatchView& bat, int32_t n, const double* x, const double* v,
                      const double* f, const uint32_t* tag, const uint8_t* type, double* bx, double* bv,
                      double* bvt, uint32_t* btag, uint8_t* btype, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (bat.kps)
        hipLaunchKernelGGL(k_vv1<true>, dim3(ceil_div(n, kBlock), 3), dim3(kBlock), 0, s, kp, bat, n, x, v, f, tag,
                           type, bx, bv, bvt, btag, btype);
    else
        hipLaunchKernelGGL(k_vv1<false>, dim3(ceil_div(n, kBlock), 3), dim3(kBlock), 0, s, kp, bat, n, x, v, f, tag,
                           type, bx, bv, bvt, btag, btype);
    return hipGetLastError();
}

hipError_t launch_sys_reduce(const BatchView& bat, int32_t n, double* v, const double* f, double half_dt,
                             const double* pe, const int32_t* npair, double* part, double* red,
                             const uint64_t* d_step, const uint64_t* base, int32_t* status, hipStream_t s)
{
    if (bat.n_sys <= 0 || bat.n_chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sys_chunks, dim3(ceil_div(bat.n_chunks, kBlock / kWave)), dim3(kBlock), 0, s, bat, n, v,
                       f, half_dt, pe, npair, part);
    hipLaunchKernelGGL(k_sys_reduce, dim3(bat.n_sys), dim3(kBlock), 0, s, bat, (const double*)part, red, d_step,
                       base, status);
    return hipGetLastError();
}

hipError_t launch_counter(uint64_t* dst, const uint64_t* src, hipStream_t s)
{
    hipLaunchKernelGGL(k_counter, dim3(1), dim3(64), 0, s, dst, src);
    return hipGetLastError();
}

hipError_t launch_sys_map(const BatchView& bat, int32_t n, uint16_t* sys_of, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sys_map, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, bat, n, sys_of);
    return hipGetLastError();
}

hipError_t launch_vv2(const KParams& kp, int32_t n, double* v, const double* f, double* red_part,
                      const double* fred_part, int32_t n_fred, double* fsum_part, hipStream_t s,
                      const DriftArgs* drift)
{
    DriftArgs dr{};
    if (drift) dr = *drift;
    hipLaunchKernelGGL(k_vv2, dim3(kRedBlocks, 3), dim3(kBlock), 0, s, kp, n, v, f, red_part, fred_part, n_fred,
                       fsum_part, dr);
    return hipGetLastError();
}

hipError_t launch_drift_skin(const KParams& kp, int32_t n, const SkinDriftArgs& d, double* red_part,
                             const double* fred_part, int32_t n_fred, double* fsum_part, hipStream_t s)
{
    hipLaunchKernelGGL(k_drift_skin, dim3(kRedBlocks), dim3(kBlock), 0, s, kp, n, d, red_part, fred_part, n_fred,
                       fsum_part);
    return hipGetLastError();
}

hipError_t launch_reduce_final(int32_t n, const double* red_part, int n_red, const double* fred_part,
                               int n_fred, double* red, double* stats, uint64_t* d_step, int32_t* status,
                               hipStream_t s, const int32_t* rebuilt, int red_stride)
{
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, s, n, red_part, n_red, red_stride, fred_part,
                       n_fred, red, stats, d_step, status, rebuilt);
    return hipGetLastError();
}

}  // namespace dpd
