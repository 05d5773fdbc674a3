// k_adjoint.hip -- vector-Jacobian product of the deterministic DPD force
// map (pair Gaussian and pair set held fixed), FP64.
//
// With F_i = sum_j f(r_ij, v_ij), f = phi e, phi = a w_C - gamma w_D u
// + sigma w_R xi / sqrt(dt), u = e.v_ij, and an upstream gradient g:
//   xbar_i = sum_j J_r^T (g_i - g_j),
//   J_r^T q = dphi/dr (e.q) e + dphi/du (e.q) (I - e e^T) v / r + phi (I - e e^T) q / r,
//   vbar_i = sum_j dphi/du (e.q) e,           dphi/du = -gamma w_D,
// and the symmetric-parameter gradients of a and gamma collect
// (g_i - g_j).w_C e and (g_i - g_j).(-w_D u e) over unordered pairs (each
// ordered pair contributes one half).  Bonds add
//   -k [ (e.q) e + (r - r0)/r (q - (e.q) e) ] to xbar.
#include "dpd_launch.h"

namespace dpd {

namespace {

__device__ __forceinline__ double weight_r(double wc, int wmode, double s)
{
    switch (wmode) {
    case 0: return sqrt(wc);
    case 1: return wc;
    case 2: return wc * wc;
    default: return pow(wc, s);
    }
}

__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double s_w[kBlock / kWave];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_down(v, d, kWave);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) s_w[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < kBlock / kWave; ++k) t += s_w[k];
    return t;
}

template <int kWMode>
__global__ __launch_bounds__(kBlock) void k_force_bwd(KParams kp, BackwardArgs a)
{
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    const int nt = kp.n_types;
    double acc_a[kMaxTypes], acc_g[kMaxTypes];
#pragma unroll
    for (int t = 0; t < kMaxTypes; ++t) { acc_a[t] = 0.0; acc_g[t] = 0.0; }
    int tyi = 0;
    if (i < a.n) {
        const int64_t N = a.n;
        const double xi = a.x[i], yi = a.x[N + i], zi = a.x[2 * N + i];
        const double vxi = a.v[i], vyi = a.v[N + i], vzi = a.v[2 * N + i];
        const double gxi = a.g[i], gyi = a.g[N + i], gzi = a.g[2 * N + i];
        const uint32_t ti = a.tag[i];
        tyi = a.type[i];
        double xb[3] = {0.0, 0.0, 0.0}, vb[3] = {0.0, 0.0, 0.0};
        if ((int64_t)a.offset[a.n] <= a.capacity) {
            for (int32_t e = a.offset[i]; e < a.offset[i + 1]; ++e) {
                const int32_t j = a.index[e];
                const double d[3] = {min_image(xi - a.x[j], kp.L[0], kp.halfL[0]),
                                     min_image(yi - a.x[N + j], kp.L[1], kp.halfL[1]),
                                     min_image(zi - a.x[2 * N + j], kp.L[2], kp.halfL[2])};
                const double r2 = dist2(d[0], d[1], d[2]);
                if (!(r2 < kp.rc2)) continue;
                const double r = sqrt(r2);
                const double e_[3] = {d[0] / r, d[1] / r, d[2] / r};
                const double vij[3] = {vxi - a.v[j], vyi - a.v[N + j], vzi - a.v[2 * N + j]};
                const double q[3] = {gxi - a.g[j], gyi - a.g[N + j], gzi - a.g[2 * N + j]};
                const int tyj = a.type[j];
                const int tp = tyi * nt + tyj;
                const double A = kp.a[tp], G = kp.g[tp], SR = kp.srdt[tp];
                const double wc = 1.0 - r * kp.inv_rc;
                const double wr = weight_r(wc, kWMode, kp.s);
                const double wd = wr * wr;
                const double dwc = -kp.inv_rc;
                const double dwr = kp.s * (wr / wc) * dwc;     // s w_C^(s-1) dw_C/dr
                const double dwd = 2.0 * wr * dwr;
                const double u = e_[0] * vij[0] + e_[1] * vij[1] + e_[2] * vij[2];
                const double xi_ij = gauss64(pair_words(ti, a.tag[j], a.step, kp.seed_lo, kp.seed_hi));
                const double phi = A * wc - G * wd * u + SR * wr * xi_ij;
                const double dphi_dr = A * dwc - G * dwd * u + SR * dwr * xi_ij;
                const double dphi_du = -G * wd;
                const double eq = e_[0] * q[0] + e_[1] * q[1] + e_[2] * q[2];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const double perp_v = (vij[k] - u * e_[k]) / r;
                    const double perp_q = (q[k] - eq * e_[k]) / r;
                    xb[k] += dphi_dr * eq * e_[k] + dphi_du * eq * perp_v + phi * perp_q;
                    vb[k] += dphi_du * eq * e_[k];
                }
                const double ca = 0.5 * wc * eq, cg = 0.5 * (-wd * u) * eq;
#pragma unroll
                for (int t = 0; t < kMaxTypes; ++t) {
                    acc_a[t] += (t == tyj) ? ca : 0.0;
                    acc_g[t] += (t == tyj) ? cg : 0.0;
                }
            }
        }
        if (kp.partner && ti < (uint32_t)a.n) {
            for (int b = 0; b < 2; ++b) {
                const int32_t pt = kp.partner[2 * (int64_t)ti + b];
                if (pt < 0 || pt >= a.n) continue;
                const int32_t j = a.idx_of_tag[pt];
                if (j < 0 || j >= a.n) continue;
                const double d[3] = {min_image(xi - a.x[j], kp.L[0], kp.halfL[0]),
                                     min_image(yi - a.x[N + j], kp.L[1], kp.halfL[1]),
                                     min_image(zi - a.x[2 * N + j], kp.L[2], kp.halfL[2])};
                const double r = sqrt(dist2(d[0], d[1], d[2]));
                const double e_[3] = {d[0] / r, d[1] / r, d[2] / r};
                const double q[3] = {gxi - a.g[j], gyi - a.g[N + j], gzi - a.g[2 * N + j]};
                const double eq = e_[0] * q[0] + e_[1] * q[1] + e_[2] * q[2];
                const double tperp = (r - kp.bond_r0) / r;
#pragma unroll
                for (int k = 0; k < 3; ++k) xb[k] += -kp.bond_k * (eq * e_[k] + tperp * (q[k] - eq * e_[k]));
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            a.xbar[k * N + i] = a.acc_xv ? a.xbar[k * N + i] + xb[k] : xb[k];
            a.vbar[k * N + i] = a.acc_xv ? a.vbar[k * N + i] + vb[k] : vb[k];
        }
    }
    // per-block partials of the type-pair matrices, row = type of i
    double* part = a.part + (int64_t)blockIdx.x * 2 * nt * nt;
    for (int tt = 0; tt < nt; ++tt)
        for (int tu = 0; tu < nt; ++tu) {
            double va = 0.0, vg = 0.0;
#pragma unroll
            for (int t = 0; t < kMaxTypes; ++t) {
                va += (t == tu) ? acc_a[t] : 0.0;
                vg += (t == tu) ? acc_g[t] : 0.0;
            }
            const bool mine = (i < a.n) && (tyi == tt);
            const double sa = block_sum(mine ? va : 0.0);
            const double sg = block_sum(mine ? vg : 0.0);
            if (threadIdx.x == 0) {
                part[tt * nt + tu] = sa;
                part[nt * nt + tt * nt + tu] = sg;
            }
        }
}

__global__ __launch_bounds__(kBlock) void k_bwd_final(int nblocks, int nt, const double* __restrict__ part,
                                                      double* __restrict__ abar, double* __restrict__ gbar,
                                                      int accumulate)
{
    __shared__ double s[kBlock];
    __shared__ double m[2 * kMaxTypes * kMaxTypes];
    const int stride = 2 * nt * nt;
    for (int c = 0; c < stride; ++c) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += kBlock) acc += part[(int64_t)b * stride + c];
        s[threadIdx.x] = acc;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) m[c] = s[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int t = 0; t < nt; ++t)
            for (int u = 0; u < nt; ++u) {
                const double va = (t == u) ? m[t * nt + t] : m[t * nt + u] + m[u * nt + t];
                const double vg = (t == u) ? m[nt * nt + t * nt + t] : m[nt * nt + t * nt + u] + m[nt * nt + u * nt + t];
                abar[t * nt + u] = accumulate ? abar[t * nt + u] + va : va;
                gbar[t * nt + u] = accumulate ? gbar[t * nt + u] + vg : vg;
            }
    }
}

}  // namespace

int backward_part_doubles(int32_t n, int32_t n_types)
{
    return ceil_div(n > 0 ? n : 1, kBlock) * 2 * n_types * n_types;
}

hipError_t launch_forces_backward(const KParams& kp, const BackwardArgs& a, hipStream_t s)
{
    const int blocks = ceil_div(a.n > 0 ? a.n : 1, kBlock);
    const dim3 grid(blocks), block(kBlock);
    switch (kp.wmode) {
    case 0: hipLaunchKernelGGL(k_force_bwd<0>, grid, block, 0, s, kp, a); break;
    case 1: hipLaunchKernelGGL(k_force_bwd<1>, grid, block, 0, s, kp, a); break;
    case 2: hipLaunchKernelGGL(k_force_bwd<2>, grid, block, 0, s, kp, a); break;
    default: hipLaunchKernelGGL(k_force_bwd<3>, grid, block, 0, s, kp, a); break;
    }
    hipLaunchKernelGGL(k_bwd_final, dim3(1), block, 0, s, blocks, kp.n_types, a.part, a.abar, a.gbar,
                       a.acc_params);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reverse of one velocity-Verlet step (lambda = 1/2).  Forward:
//   v_h = v + c F,  x' = x + dt v_h (wrapped),  F' = Phi(x', v_h),
//   v' = v_h + c F',  c = dt/2,  then the reorder x'_new[q] = x'_old[perm[q]].
// Reverse, with incoming adjoints (xb', vb', Fb') of the new state:
//   Fb'  += c vb'                           (k_bwd_prep)
//   (xPhi, vPhi) = VJP of Phi at (x', v_h)  (k_force_bwd)
//   xt = xb' + xPhi,  vh = vb' + vPhi + dt xt
//   xb[perm[q]] = xt,  vb[perm[q]] = vh,  Fb[perm[q]] = c vh   (k_bwd_scatter)
// v_h is recovered as v' - c F' (within rounding of the forward value).
// ---------------------------------------------------------------------------

namespace {

__global__ __launch_bounds__(kBlock) void k_bwd_prep(KParams kp, int32_t n, const double* __restrict__ v,
                                                     const double* __restrict__ f,
                                                     const double* __restrict__ gv_in,
                                                     const double* __restrict__ gf_in, double* __restrict__ vt,
                                                     double* __restrict__ gf_eff)
{
    const int64_t a = (int64_t)blockIdx.y * n + blockIdx.x * kBlock + threadIdx.x;
    if (blockIdx.x * kBlock + threadIdx.x >= n) return;
    vt[a] = __fma_rn(-kp.half_dt, f[a], v[a]);
    gf_eff[a] = __fma_rn(kp.half_dt, gv_in[a], gf_in[a]);
}

__global__ __launch_bounds__(kBlock) void k_bwd_scatter(KParams kp, int32_t n, const int32_t* __restrict__ perm,
                                                        const double* __restrict__ gx_in,
                                                        const double* __restrict__ gv_in,
                                                        const double* __restrict__ xphi,
                                                        const double* __restrict__ vphi,
                                                        double* __restrict__ gx_out, double* __restrict__ gv_out,
                                                        double* __restrict__ gf_out)
{
    const int32_t q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    const int64_t base = (int64_t)blockIdx.y * n;
    const int64_t src = base + q, dst = base + perm[q];
    const double xt = gx_in[src] + xphi[src];
    const double vh = __fma_rn(kp.dt, xt, gv_in[src] + vphi[src]);
    gx_out[dst] = xt;
    gv_out[dst] = vh;
    gf_out[dst] = kp.half_dt * vh;
}

}  // namespace

hipError_t launch_step_backward(const KParams& kp, const StepBackwardArgs& b, hipStream_t s)
{
    const int32_t n = b.fwd.n;
    if (n <= 0) return hipSuccess;
    const dim3 grid(ceil_div(n, kBlock), 3), block(kBlock);
    hipLaunchKernelGGL(k_bwd_prep, grid, block, 0, s, kp, n, b.v_new, b.f_new, b.gv_in, b.gf_in, b.vt, b.gf_eff);
    BackwardArgs a = b.fwd;
    a.v = b.vt;
    a.g = b.gf_eff;
    a.xbar = b.xphi;
    a.vbar = b.vphi;
    a.acc_xv = 0;
    a.acc_params = 1;
    hipError_t e = launch_forces_backward(kp, a, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bwd_scatter, grid, block, 0, s, kp, n, b.perm, b.gx_in, b.gv_in, b.xphi, b.vphi, b.gx_out,
                       b.gv_out, b.gf_out);
    return hipGetLastError();
}

}  // namespace dpd
