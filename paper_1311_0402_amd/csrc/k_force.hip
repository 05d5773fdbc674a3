// k_force.hip -- pairwise DPD force (Sec. 2, Eqs (2)-(8) of the paper),
// harmonic bonds (Sec. 4.5) and the reverse-Poiseuille body force (Sec. 4.2).
//
// One lane per particle i walks i's ascending neighbour row.  Per pair:
// minimum-image separation, w_C = 1 - r/r_c, w_R = w_C^s (specialised for
// s = 1/2, 1, 2), w_D = w_R^2, the symmetric pair Gaussian xi_ij from
// Philox4x32-10 on (min tag, max tag, step, seed) and Box-Muller, and
// phi = a w_C - gamma w_D (e.v_ij) + sigma w_R xi / sqrt(dt); F_i += phi e.
// The same pair seen from j gives bitwise the negated contribution.
//
// FP64 form: everything in double.  Mixed form: separations from FP32
// offsets inside each particle's cell plus the cell difference times the
// FP32 cell length, FP32 pair arithmetic with hardware rsqrt / sqrt / log /
// cos, and per-particle compensated (two-sum) FP32 accumulation; the
// result is stored as FP64.
#include "dpd_launch.h"

namespace dpd {

namespace {

constexpr int kTab = kMaxTypes * kMaxTypes;
// below this squared separation (r < 0.01 r_c-units) the mixed kernel takes
// the pair's geometry from the FP64 positions
constexpr float kCloseR2 = 1.0e-4f;

__device__ __forceinline__ double weight_r(double wc, int wmode, double s)
{
    switch (wmode) {
    case 0: return sqrt(wc);
    case 1: return wc;
    case 2: return wc * wc;
    default: return pow(wc, s);
    }
}

// FP32 weight: hardware sqrt, or 2^(s log2 w_C) for a general exponent
__device__ __forceinline__ float weight_r32(float wc, int wmode, float s)
{
    switch (wmode) {
    case 0: return sqrtf(wc);
    case 1: return wc;
    case 2: return wc * wc;
    default: return wc > 0.f ? exp2f(s * __log2f(wc)) : 0.f;
    }
}

// block sum of two doubles into part[blockIdx.x * 2 + {0,1}] (fixed order)
__device__ __forceinline__ void block_partials2(double a, double b, double* __restrict__ part)
{
    __shared__ double s_a[kBlock / kWave], s_b[kBlock / kWave];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        a += __shfl_down(a, d, kWave);
        b += __shfl_down(b, d, kWave);
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) { s_a[w] = a; s_b[w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
        for (int k = 0; k < kBlock / kWave; ++k) { ta += s_a[k]; tb += s_b[k]; }
        part[2 * blockIdx.x] = ta;
        part[2 * blockIdx.x + 1] = tb;
    }
}

// bonds and body force, shared by both precisions (FP64)
__device__ __forceinline__ void add_bonds_body(const KParams& kp, const ForceArgs& a, int32_t i,
                                               double xi, double yi, double zi, double& fx, double& fy,
                                               double& fz, double& pe)
{
    const int64_t N = a.n;
    if (kp.partner && a.tag[i] < (uint32_t)a.n) {
        const uint32_t t = a.tag[i];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int32_t pt = kp.partner[2 * (int64_t)t + b];
            if (pt < 0) continue;
            const int32_t j = (pt < a.n) ? a.idx_of_tag[pt] : -1;
            if (j < 0 || j >= a.n) {
                if (a.status) atomicOr(a.status, 4 /* DPD_STATUS_BAD_BOND */);
                continue;
            }
            const double dx = min_image(xi - a.x[j], kp.L[0], kp.halfL[0]);
            const double dy = min_image(yi - a.x[N + j], kp.L[1], kp.halfL[1]);
            const double dz = min_image(zi - a.x[2 * N + j], kp.L[2], kp.halfL[2]);
            const double r = sqrt(dist2(dx, dy, dz));
            const double ext = r - kp.bond_r0;
            const double mag = -kp.bond_k * ext;
            fx += mag * dx / r;
            fy += mag * dy / r;
            fz += mag * dz / r;
            pe += 0.25 * kp.bond_k * ext * ext;
        }
    }
    if (kp.body_g != 0.0) fx += (yi < kp.body_split) ? kp.body_g : -kp.body_g;
}

template <int kWMode>
__global__ __launch_bounds__(kBlock) void k_force_fp64(KParams kp, ForceArgs a)
{
    __shared__ double s_a[kTab], s_g[kTab], s_s[kTab];
    const int nt2 = kp.n_types * kp.n_types;
    for (int t = threadIdx.x; t < nt2; t += kBlock) {
        s_a[t] = kp.a[t]; s_g[t] = kp.g[t]; s_s[t] = kp.srdt[t];
    }
    __syncthreads();
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    double fx = 0.0, fy = 0.0, fz = 0.0, pe = 0.0, npair = 0.0;
    if (i < a.n) {
        const int64_t N = a.n;
        const uint64_t step = (a.d_step ? *a.d_step : 0ull) + a.step_add;
        const double xi = a.x[i], yi = a.x[N + i], zi = a.x[2 * N + i];
        const double vxi = a.v[i], vyi = a.v[N + i], vzi = a.v[2 * N + i];
        const uint32_t ti = a.tag[i];
        const int tyi = a.type[i] * kp.n_types;
        if ((int64_t)a.offset[a.n] <= a.capacity) {
            const int32_t e1 = a.offset[i + 1];
            for (int32_t e = a.offset[i]; e < e1; ++e) {
                const int32_t j = a.index[e];
                const double dx = min_image(xi - a.x[j], kp.L[0], kp.halfL[0]);
                const double dy = min_image(yi - a.x[N + j], kp.L[1], kp.halfL[1]);
                const double dz = min_image(zi - a.x[2 * N + j], kp.L[2], kp.halfL[2]);
                const double r2 = dist2(dx, dy, dz);
                if (!(r2 < kp.rc2)) continue;
                const double r = sqrt(r2);
                const double ex = dx / r, ey = dy / r, ez = dz / r;
                const double wc = 1.0 - r * kp.inv_rc;
                const double wr = weight_r(wc, kWMode, kp.s);
                const double wd = wr * wr;
                const double ev = ex * (vxi - a.v[j]) + ey * (vyi - a.v[N + j]) + ez * (vzi - a.v[2 * N + j]);
                const int tp = tyi + a.type[j];
                const double xi_ij = gauss64(pair_words(ti, a.tag[j], step, kp.seed_lo, kp.seed_hi));
                const double phi = s_a[tp] * wc - s_g[tp] * wd * ev + s_s[tp] * wr * xi_ij;
                fx += phi * ex;
                fy += phi * ey;
                fz += phi * ez;
                pe += 0.25 * s_a[tp] * kp.r_c * wc * wc;
                npair += 1.0;
            }
        }
        add_bonds_body(kp, a, i, xi, yi, zi, fx, fy, fz, pe);
        a.f[i] = fx;
        a.f[N + i] = fy;
        a.f[2 * N + i] = fz;
        if (a.pe) a.pe[i] = pe;
    }
    if (a.fred_part) block_partials2(pe, 0.5 * npair, a.fred_part);
}

__device__ __forceinline__ void two_sum_add(float& s, float& c, float v)
{
    const float t = s + v;
    const float z = t - s;
    c += (s - (t - z)) + (v - z);
    s = t;
}

__device__ __forceinline__ int cell_delta(int32_t ci, int32_t cj, int32_t n)
{
    int d = ci - cj;
    d = d > 1 ? d - n : d;
    return d < -1 ? d + n : d;
}

template <int kWMode>
__global__ __launch_bounds__(kBlock) void k_force_mixed(KParams kp, ForceArgs a)
{
    __shared__ float s_a[kTab], s_g[kTab], s_s[kTab];
    const int nt2 = kp.n_types * kp.n_types;
    for (int t = threadIdx.x; t < nt2; t += kBlock) {
        s_a[t] = (float)kp.a[t]; s_g[t] = (float)kp.g[t]; s_s[t] = (float)kp.srdt[t];
    }
    __syncthreads();
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    double pe64 = 0.0, npair = 0.0;
    if (i < a.n) {
        const int64_t N = a.n;
        const uint64_t step = (a.d_step ? *a.d_step : 0ull) + a.step_add;
        const float xi = a.x32[i], yi = a.x32[N + i], zi = a.x32[2 * N + i];
        const float vxi = a.v32[i], vyi = a.v32[N + i], vzi = a.v32[2 * N + i];
        const uint32_t ci = a.cell_xyz[i];
        const int32_t cix = ci & 1023u, ciy = (ci >> 10) & 1023u, ciz = ci >> 20;
        const uint32_t ti = a.tag[i];
        const int tyi = a.type[i] * kp.n_types;
        const float rc32 = (float)kp.r_c, inv_rc32 = (float)kp.inv_rc, rc2_32 = (float)kp.rc2;
        float sx = 0.f, sy = 0.f, sz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f, pe = 0.f;
        if ((int64_t)a.offset[a.n] <= a.capacity) {
            const int32_t e1 = a.offset[i + 1];
            for (int32_t e = a.offset[i]; e < e1; ++e) {
                const int32_t j = a.index[e];
                const uint32_t cj = a.cell_xyz[j];
                const float ox = (float)cell_delta(cix, (int32_t)(cj & 1023u), kp.nc[0]) * kp.cell_len32[0];
                const float oy = (float)cell_delta(ciy, (int32_t)((cj >> 10) & 1023u), kp.nc[1]) * kp.cell_len32[1];
                const float oz = (float)cell_delta(ciz, (int32_t)(cj >> 20), kp.nc[2]) * kp.cell_len32[2];
                const float dx = (xi - a.x32[j]) + ox;
                const float dy = (yi - a.x32[N + j]) + oy;
                const float dz = (zi - a.x32[2 * N + j]) + oz;
                const float r2 = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
                // with no skin the FP64 list already decided the pair set; a
                // skin needs the FP32 test (documented reading)
                if (kp.rl2 != kp.rc2 && !(r2 < rc2_32)) continue;
                float r, ex, ey, ez;
                if (r2 >= kCloseR2) {
                    const float inv_r = rsqrtf(r2);
                    r = r2 * inv_r;
                    ex = dx * inv_r; ey = dy * inv_r; ez = dz * inv_r;
                } else {
                    // FP32 offsets cannot resolve the direction of a nearly
                    // coincident pair: take its geometry from FP64 positions
                    const double ddx = min_image(a.x[i] - a.x[j], kp.L[0], kp.halfL[0]);
                    const double ddy = min_image(a.x[N + i] - a.x[N + j], kp.L[1], kp.halfL[1]);
                    const double ddz = min_image(a.x[2 * N + i] - a.x[2 * N + j], kp.L[2], kp.halfL[2]);
                    const double rr = sqrt(dist2(ddx, ddy, ddz));
                    if (!(rr > 0.0)) continue;      // coincident: no direction, no force
                    r = (float)rr;
                    ex = (float)(ddx / rr); ey = (float)(ddy / rr); ez = (float)(ddz / rr);
                }
                float wc = 1.0f - r * inv_rc32;
                wc = wc > 0.f ? wc : 0.f;
                const float wr = weight_r32(wc, kWMode, (float)kp.s);
                const float wd = wr * wr;
                const float ev = ex * (vxi - a.v32[j]) + ey * (vyi - a.v32[N + j]) + ez * (vzi - a.v32[2 * N + j]);
                const int tp = tyi + a.type[j];
                const float xi_ij = gauss32(pair_words(ti, a.tag[j], step, kp.seed_lo, kp.seed_hi));
                const float phi = s_a[tp] * wc - s_g[tp] * wd * ev + s_s[tp] * wr * xi_ij;
                two_sum_add(sx, cx, phi * ex);
                two_sum_add(sy, cy, phi * ey);
                two_sum_add(sz, cz, phi * ez);
                pe += 0.25f * s_a[tp] * rc32 * wc * wc;
                npair += 1.0;
            }
        }
        double fx = (double)sx + (double)cx, fy = (double)sy + (double)cy, fz = (double)sz + (double)cz;
        pe64 = pe;
        if (kp.partner || kp.body_g != 0.0)
            add_bonds_body(kp, a, i, a.x[i], a.x[N + i], a.x[2 * N + i], fx, fy, fz, pe64);
        a.f[i] = fx;
        a.f[N + i] = fy;
        a.f[2 * N + i] = fz;
        if (a.pe) a.pe[i] = pe64;
    }
    if (a.fred_part) block_partials2(pe64, 0.5 * npair, a.fred_part);
}

}  // namespace

int force_blocks(int32_t n) { return ceil_div(n > 0 ? n : 1, kBlock); }

hipError_t launch_forces(const KParams& kp, int precision, const ForceArgs& a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const dim3 grid(force_blocks(a.n)), block(kBlock);
    if (precision == 0) {
        switch (kp.wmode) {
        case 0: hipLaunchKernelGGL(k_force_fp64<0>, grid, block, 0, s, kp, a); break;
        case 1: hipLaunchKernelGGL(k_force_fp64<1>, grid, block, 0, s, kp, a); break;
        case 2: hipLaunchKernelGGL(k_force_fp64<2>, grid, block, 0, s, kp, a); break;
        default: hipLaunchKernelGGL(k_force_fp64<3>, grid, block, 0, s, kp, a); break;
        }
    } else {
        switch (kp.wmode) {
        case 0: hipLaunchKernelGGL(k_force_mixed<0>, grid, block, 0, s, kp, a); break;
        case 1: hipLaunchKernelGGL(k_force_mixed<1>, grid, block, 0, s, kp, a); break;
        case 2: hipLaunchKernelGGL(k_force_mixed<2>, grid, block, 0, s, kp, a); break;
        default: hipLaunchKernelGGL(k_force_mixed<3>, grid, block, 0, s, kp, a); break;
        }
    }
    return hipGetLastError();
}

}  // namespace dpd
