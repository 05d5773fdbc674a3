// k_numerics.hip -- the paper's numerics as A/B variants of the pair
// Gaussian and of the power function (Sec. 3.5, Algorithms 4 and 5, Table
// 3), written from the mathematics and measured beside the device library.
//
// * TEA (Wheeler & Needham's tiny encryption algorithm) on per-particle
//   signatures: a signature blends the bit-reversed tag with the leading
//   mantissa bits of the three velocity components through 16 TEA rounds
//   and xors the two halves; a pair's two 32-bit words are 4 TEA rounds on
//   (smaller signature, larger signature).  The keys are (seed low, seed
//   high, step low, step high); the round constant is TEA's own.
// * fast_log2: exponent from the bits, mantissa folded into
//   [sqrt(1/2), sqrt(2)), log2 m = (2 / ln 2) atanh(z), z = (m - 1) / (m + 1),
//   by the odd power series of atanh (|z| <= 0.1716, eleven terms).
// * fast_cos2pi: cos(2 pi u) for u in [0, 1): folded by the symmetries of
//   the cosine into an angle x in [0, pi/4] where either cos x or sin x is
//   wanted, each by its power series (no branches: both series run).
// * fast_pow: a^b = 2^N 2^r, N the integer nearest b log2 a and r the rest,
//   formed with fused multiply-adds so its absolute error stays near one
//   ulp of 1; 2^r by the power series of exp(r ln 2) on |r| <= 1/2.
//
// Microbenchmarks: one wave's dependent chain of a function (cycles per
// evaluation, from the shader clock), and whole-grid throughput of pair
// Gaussians from each generator.
#include "dpd_launch.h"

namespace dpd {

namespace {

constexpr uint32_t kTeaDelta = 0x9E3779B9u;    // TEA's round constant

struct TeaKey {
    uint32_t k0, k1, k2, k3;
};

__device__ __forceinline__ void tea(int rounds, uint32_t& v0, uint32_t& v1, const TeaKey& k)
{
    uint32_t sum = 0;
    for (int r = 0; r < rounds; ++r) {
        sum += kTeaDelta;
        v0 += ((v1 << 4) + k.k0) ^ (v1 + sum) ^ ((v1 >> 5) + k.k1);
        v1 += ((v0 << 4) + k.k2) ^ (v0 + sum) ^ ((v0 >> 5) + k.k3);
    }
}

__device__ __forceinline__ TeaKey tea_key(uint64_t seed, uint64_t step)
{
    return TeaKey{(uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)step, (uint32_t)(step >> 32)};
}

// the leading 11 bits of a double's 52-bit mantissa
__device__ __forceinline__ uint32_t mantissa11(double v)
{
    return (uint32_t)((uint64_t)__double_as_longlong(v) >> 41) & 0x7FFu;
}

// bits of bx, by, bz interleaved (x lowest), 33 bits kept to the low 32
__device__ __forceinline__ uint32_t interleave3(uint32_t bx, uint32_t by, uint32_t bz)
{
    uint32_t out = 0;
#pragma unroll
    for (int b = 0; b < 11; ++b) {
        out |= ((bx >> b) & 1u) << (3 * b);
        if (3 * b + 1 < 32) out |= ((by >> b) & 1u) << (3 * b + 1);
        if (3 * b + 2 < 32) out |= ((bz >> b) & 1u) << (3 * b + 2);
    }
    return out;
}

__device__ __forceinline__ uint32_t signature(uint32_t tag, double vx, double vy, double vz, const TeaKey& k)
{
    uint32_t v0 = __brev(tag);
    uint32_t v1 = interleave3(mantissa11(vx), mantissa11(vy), mantissa11(vz));
    tea(16, v0, v1, k);
    return v0 ^ v1;
}

__device__ __forceinline__ void pair_tea_words(uint32_t si, uint32_t sj, const TeaKey& k, uint32_t& w0, uint32_t& w1)
{
    w0 = si < sj ? si : sj;
    w1 = si < sj ? sj : si;
    tea(4, w0, w1, k);
}

// 1 / d by the hardware reciprocal estimate (about 2^-24 relative) and two
// Newton steps (each squares the relative error: 2^-48, then rounding)
__device__ __forceinline__ double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = __fma_rn(r, __fma_rn(-d, r, 1.0), r);
    return __fma_rn(r, __fma_rn(-d, r, 1.0), r);
}

// log2 a for a positive normal double
__device__ __forceinline__ void fast_log2_split(double a, double& e_out, double& f_out)
{
    constexpr double kRt2 = 1.41421356237309504880;
    // 2 / ((2k + 1) ln 2), k = 0 .. 10
    constexpr double c[11] = {2.0 / 0.69314718055994530942,       2.0 / (3.0 * 0.69314718055994530942),
                              2.0 / (5.0 * 0.69314718055994530942),  2.0 / (7.0 * 0.69314718055994530942),
                              2.0 / (9.0 * 0.69314718055994530942),  2.0 / (11.0 * 0.69314718055994530942),
                              2.0 / (13.0 * 0.69314718055994530942), 2.0 / (15.0 * 0.69314718055994530942),
                              2.0 / (17.0 * 0.69314718055994530942), 2.0 / (19.0 * 0.69314718055994530942),
                              2.0 / (21.0 * 0.69314718055994530942)};
    const uint64_t bits = (uint64_t)__double_as_longlong(a);
    int e = (int)((bits >> 52) & 0x7FF) - 1023;
    double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    const bool hi = m > kRt2;
    m = hi ? 0.5 * m : m;
    e = hi ? e + 1 : e;
    const double z = (m - 1.0) * recip(m + 1.0);
    const double z2 = z * z;
    double p = c[10];
#pragma unroll
    for (int k = 9; k >= 0; --k) p = __fma_rn(p, z2, c[k]);
    e_out = (double)e;
    f_out = z * p;
}

__device__ __forceinline__ double fast_log2(double a)
{
    double e, f;
    fast_log2_split(a, e, f);
    return e + f;
}

__device__ __forceinline__ double fast_ln(double a) { return 0.69314718055994530942 * fast_log2(a); }

// cos x and sin x on |x| <= pi/4 by their power series
__device__ __forceinline__ double cos_series(double x2)
{
    // (-1)^k / (2k)!, k = 0 .. 9
    constexpr double c[10] = {1.0, -1.0 / 2.0, 1.0 / 24.0, -1.0 / 720.0, 1.0 / 40320.0, -1.0 / 3628800.0,
                              1.0 / 479001600.0, -1.0 / 87178291200.0, 1.0 / 20922789888000.0,
                              -1.0 / 6402373705728000.0};
    double p = c[9];
#pragma unroll
    for (int k = 8; k >= 0; --k) p = __fma_rn(p, x2, c[k]);
    return p;
}

__device__ __forceinline__ double sin_series(double x, double x2)
{
    // (-1)^k / (2k + 1)!, k = 0 .. 9
    constexpr double c[10] = {1.0, -1.0 / 6.0, 1.0 / 120.0, -1.0 / 5040.0, 1.0 / 362880.0, -1.0 / 39916800.0,
                              1.0 / 6227020800.0, -1.0 / 1307674368000.0, 1.0 / 355687428096000.0,
                              -1.0 / 121645100408832000.0};
    double p = c[9];
#pragma unroll
    for (int k = 8; k >= 0; --k) p = __fma_rn(p, x2, c[k]);
    return x * p;
}

// cos(2 pi u), u in [0, 1)
__device__ __forceinline__ double fast_cos2pi(double u)
{
    constexpr double kTwoPi = 6.28318530717958647693;
    const double v = u > 0.5 ? 1.0 - u : u;            // cos(2 pi u) = cos(2 pi (1 - u)); v in [0, 1/2]
    const bool back = v > 0.25;                        // cos(2 pi v) = -cos(2 pi (1/2 - v))
    const double w = back ? 0.5 - v : v;               // [0, 1/4]
    const bool use_sin = w > 0.125;                    // cos(2 pi w) = sin(2 pi (1/4 - w))
    const double x = kTwoPi * (use_sin ? 0.25 - w : w);  // [0, pi/4]
    const double x2 = x * x;
    const double c = use_sin ? sin_series(x, x2) : cos_series(x2);
    return back ? -c : c;
}

// a^b for a > 0 (normal), b finite, the result in the normal range
__device__ __forceinline__ double fast_pow(double a, double b)
{
    // (ln 2)^k / k!, k = 0 .. 14
    constexpr double kLn2 = 0.69314718055994530942;
    constexpr double c[15] = {1.0,
                              kLn2,
                              kLn2 * kLn2 / 2.0,
                              kLn2 * kLn2 * kLn2 / 6.0,
                              kLn2 * kLn2 * kLn2 * kLn2 / 24.0,
                              kLn2 * kLn2 * kLn2 * kLn2 * kLn2 / 120.0,
                              kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 / 720.0,
                              kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 / 5040.0,
                              kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 / 40320.0,
                              kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 / 362880.0,
                              kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 / 3628800.0,
                              kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 / 39916800.0,
                              kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 /
                                  479001600.0,
                              kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 *
                                  kLn2 / 6227020800.0,
                              kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 * kLn2 *
                                  kLn2 * kLn2 / 87178291200.0};
    double e, f;
    fast_log2_split(a, e, f);                          // log2 a = e + f, |f| <= 1/2
    const double n = rint(b * (e + f));
    const double r = __fma_rn(b, f, __fma_rn(b, e, -n));   // b (e + f) - n, one rounding per step
    double p = c[14];
#pragma unroll
    for (int k = 13; k >= 0; --k) p = __fma_rn(p, r, c[k]);
    return __builtin_amdgcn_ldexp(p, (int)n);
}

__device__ __forceinline__ double eval_fn(int fn, double a, double b)
{
    switch (fn) {
    case DPD_FN_LOG: return log(a);
    case DPD_FN_FASTLOG: return fast_ln(a);
    case DPD_FN_COS2PI: return cospi(2.0 * a);
    case DPD_FN_FASTCOS2PI: return fast_cos2pi(a);
    case DPD_FN_POW: return pow(a, b);
    default: return fast_pow(a, b);
    }
}

__global__ __launch_bounds__(kBlock) void k_numerics_eval(int fn, int64_t n, const double* __restrict__ a,
                                                          const double* __restrict__ b, double* __restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        out[i] = eval_fn(fn, a[i], b ? b[i] : 0.0);
}

// One wave: each lane runs a chain of `chain` dependent evaluations; the
// next argument is an affine map of the previous result that keeps it in
// the function's domain.  cycles[0] = shader clock ticks of the chain.
template <int kFn>
__global__ __launch_bounds__(kWave) void k_numerics_latency(int32_t chain, int64_t* __restrict__ cycles,
                                                            double* __restrict__ sink)
{
    double x = 0.3 + 0.001 * threadIdx.x;
    __syncthreads();
    const int64_t t0 = clock64();
    for (int32_t k = 0; k < chain; ++k) {
        const double y = eval_fn(kFn, x, 0.75 + 0.25 * x);
        // log: y in about [-5, 0] -> x in [0.25, 0.5]; cos: y in [-1, 1] -> x in
        // [0.25, 0.75]; pow: y in (0, 1) -> x in (0.25, 0.5)
        x = kFn <= DPD_FN_FASTLOG ? __fma_rn(y, 0.05, 0.5) : __fma_rn(y, 0.25, 0.5);
        x = x > 0.999 ? 0.999 : (x < 0.001 ? 0.001 : x);
    }
    const int64_t t1 = clock64();
    if (threadIdx.x == 0) cycles[0] = t1 - t0;
    sink[threadIdx.x] = x;
}

// Pair Gaussians of consecutive pairs (t, t + 1 .. t + m) of each thread's
// tag t: generator 0 = Philox4x32-10 words and Box-Muller with the device
// library's log, sqrt and cospi (the FP64 force pass's generator);
// generator 1 = TEA-4 on signatures with fast_ln and fast_cos2pi.
// Signatures of generator 1 come from sig[] (one per tag).
template <int kGen>
__global__ __launch_bounds__(kBlock) void k_gauss_throughput(int32_t n_tags, int32_t pairs_per_thread, uint64_t step,
                                                             uint64_t seed, const uint32_t* __restrict__ sig,
                                                             double* __restrict__ sink)
{
    const int32_t t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n_tags) return;
    const TeaKey key = tea_key(seed, step);
    double acc = 0.0;
    const uint32_t st = kGen == 1 ? sig[t] : 0u;
    for (int32_t m = 1; m <= pairs_per_thread; ++m) {
        int32_t j = t + m;
        j = j >= n_tags ? j - n_tags : j;
        double z;
        if constexpr (kGen == 0) {
            z = gauss64(pair_words((uint32_t)t, (uint32_t)j, step, (uint32_t)seed, (uint32_t)(seed >> 32)));
        } else {
            uint32_t w0, w1;
            pair_tea_words(st, sig[j], key, w0, w1);
            const double u1 = ((double)w0 + 0.5) * 0x1p-32;
            const double u2 = (double)w1 * 0x1p-32;
            z = sqrt(-2.0 * fast_ln(u1)) * fast_cos2pi(u2);
        }
        acc += z;
    }
    sink[t] = acc;
}

__global__ __launch_bounds__(kBlock) void k_signatures(int32_t n, const uint32_t* __restrict__ tag,
                                                       const double* __restrict__ v, uint64_t step, uint64_t seed,
                                                       uint32_t* __restrict__ sig)
{
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t N = n;
    sig[i] = signature(tag[i], v[i], v[N + i], v[2 * N + i], tea_key(seed, step));
}

// xi of listed pairs from signatures: w (nullable) gets the two TEA words
__global__ __launch_bounds__(kBlock) void k_tea_gauss(int64_t n, const uint32_t* __restrict__ si,
                                                      const uint32_t* __restrict__ sj, uint64_t step, uint64_t seed,
                                                      uint32_t* __restrict__ w, double* __restrict__ xi)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    uint32_t w0, w1;
    pair_tea_words(si[i], sj[i], tea_key(seed, step), w0, w1);
    if (w) { w[2 * i] = w0; w[2 * i + 1] = w1; }
    const double u1 = ((double)w0 + 0.5) * 0x1p-32;
    const double u2 = (double)w1 * 0x1p-32;
    xi[i] = sqrt(-2.0 * fast_ln(u1)) * fast_cos2pi(u2);
}

int grid_for(int64_t n)
{
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

hipError_t launch_numerics_eval(int fn, int64_t n, const double* a, const double* b, double* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_numerics_eval, dim3(grid_for(n)), dim3(kBlock), 0, s, fn, n, a, b, out);
    return hipGetLastError();
}

hipError_t launch_numerics_latency(int fn, int32_t chain, int64_t* cycles, double* sink, hipStream_t s)
{
    switch (fn) {
#define DPD_LAT(F) \
    case F: hipLaunchKernelGGL(k_numerics_latency<F>, dim3(1), dim3(kWave), 0, s, chain, cycles, sink); break;
    DPD_LAT(DPD_FN_LOG)
    DPD_LAT(DPD_FN_FASTLOG)
    DPD_LAT(DPD_FN_COS2PI)
    DPD_LAT(DPD_FN_FASTCOS2PI)
    DPD_LAT(DPD_FN_POW)
    DPD_LAT(DPD_FN_FASTPOW)
#undef DPD_LAT
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_signatures(int32_t n, const uint32_t* tag, const double* v, uint64_t step, uint64_t seed,
                             uint32_t* sig, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_signatures, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, n, tag, v, step, seed, sig);
    return hipGetLastError();
}

hipError_t launch_tea_gauss(int64_t n, const uint32_t* si, const uint32_t* sj, uint64_t step, uint64_t seed,
                            uint32_t* w, double* xi, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tea_gauss, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, n, si, sj, step, seed, w, xi);
    return hipGetLastError();
}

hipError_t launch_gauss_throughput(int gen, int32_t n_tags, int32_t pairs_per_thread, uint64_t step, uint64_t seed,
                                   const uint32_t* sig, double* sink, hipStream_t s)
{
    if (n_tags <= 0) return hipSuccess;
    if (gen == 0)
        hipLaunchKernelGGL(k_gauss_throughput<0>, dim3(ceil_div(n_tags, kBlock)), dim3(kBlock), 0, s, n_tags,
                           pairs_per_thread, step, seed, sig, sink);
    else
        hipLaunchKernelGGL(k_gauss_throughput<1>, dim3(ceil_div(n_tags, kBlock)), dim3(kBlock), 0, s, n_tags,
                           pairs_per_thread, step, seed, sig, sink);
    return hipGetLastError();
}

}  // namespace dpd
