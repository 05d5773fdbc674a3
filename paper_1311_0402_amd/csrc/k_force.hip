// k_force.hip -- pairwise DPD force (Sec. 2, Eqs (2)-(8) of the paper),
// harmonic bonds (Sec. 4.5) and the reverse-Poiseuille body force (Sec. 4.2).
//
// Per pair (the lane layout is described at the kernels below):
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
#include <atomic>

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

// FP32 weight: hardware square root (v_sqrt_f32, within an ulp), or
// 2^(s log2 w_C) for a general exponent
__device__ __forceinline__ float weight_r32(float wc, int wmode, float s)
{
    switch (wmode) {
    case 0: return __builtin_amdgcn_sqrtf(wc);
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

// The step's second half-kick for row i, in the force pass's row epilogue
// (single systems): v = fma(dt/2, F, v_h) with v_h from a.vv_v, then with a
// drift the next step's first half-kick and drift into the reorder's source
// arrays, else v stored back; the arithmetic of k_vv2 with its drift, so the
// state is the same bit for bit.  acc: this lane's momentum and |v|^2
// accumulators (LDS, component k at acc[2k kBlock] and acc[(2k+1) kBlock]).
// The row's operands of the half-kick (v_h and x, tag and type for the
// drift), requested when the pass starts the row's chunk so their latency
// hides behind the chunk's pairs.
struct VVIn {
    double v[3], x[3];
    uint32_t tag;
    uint8_t type;
};

__device__ __forceinline__ VVIn vv_load(const ForceArgs& a, int64_t N, int32_t i)
{
    VVIn o;
    const DriftArgs& dr = a.vv_drift;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        o.v[k] = a.vv_v[k * N + i];
        o.x[k] = dr.bx ? dr.x[k * N + i] : 0.0;
    }
    o.tag = dr.bx ? dr.tag[i] : 0u;
    o.type = dr.bx ? dr.type[i] : (uint8_t)0;
    return o;
}

__device__ __forceinline__ void vv_row(const KParams& kp, const ForceArgs& a, int64_t N, int32_t i, const VVIn& in,
                                       double fx, double fy, double fz, double* __restrict__ acc)
{
    const DriftArgs& dr = a.vv_drift;
    const double fk[3] = {fx, fy, fz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int64_t o = k * N + i;
        const double vn = __fma_rn(kp.half_dt, fk[k], in.v[k]);
        if (dr.bx) {
            const double vh = __fma_rn(kp.half_dt, fk[k], vn);
            double xn = __fma_rn(kp.dt, vh, in.x[k]);
            if (xn < 0.0) xn = xn + kp.L[k];
            if (xn >= kp.L[k]) xn = xn - kp.L[k];
            dr.bx[o] = xn;
            dr.bv[o] = vh;
            if (dr.bvt) dr.bvt[o] = __fma_rn(kp.lam_dt, fk[k], vn);
        } else {
            a.vv_v[o] = vn;
        }
        acc[2 * k * kBlock] += vn;
        acc[(2 * k + 1) * kBlock] += vn * vn;
    }
    if (dr.bx) {
        dr.btag[i] = in.tag;
        dr.btype[i] = in.type;
    }
}

// the workgroup's momentum and |v|^2 partials from the lanes' accumulators
// (fixed order), into part[k][blockIdx][0..1] with stride gridDim.x
__device__ __forceinline__ void vv_partials(const double* __restrict__ s_acc, double* __restrict__ part)
{
    __syncthreads();
    if (threadIdx.x < 6) {
        const double* src = s_acc + threadIdx.x * kBlock;
        double t = 0.0;
        for (int m = 0; m < kBlock; ++m) t += src[m];
        const int k = threadIdx.x >> 1;
        part[2 * ((int64_t)k * gridDim.x + blockIdx.x) + (threadIdx.x & 1)] = t;
    }
}

// bonds and body force, shared by both precisions (FP64)
__device__ __forceinline__ void add_bonds_body(const KParams& kp, const ForceArgs& a, int32_t i,
                                               double xi, double yi, double zi, double& fx, double& fy,
                                               double& fz, double& pe)
{
    const int64_t N = a.n;
    if (kp.partner && (a.pidx || a.tag[i] < (uint32_t)a.n)) {
        const uint32_t t = a.pidx ? 0u : a.tag[i];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            int32_t j;
            if (a.pidx) {
                j = a.pidx[2 * (int64_t)i + b];
                if (j == -1) continue;
            } else {
                const int32_t pt = kp.partner[2 * (int64_t)t + b];
                if (pt < 0) continue;
                j = (pt < a.n) ? a.idx_of_tag[pt] : -1;
            }
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

// Work layout.  A wavefront owns 64 consecutive particles ("rows"); their
// neighbour rows are one contiguous run of CSR entries, which the wave walks
// 64 entries at a time, one pair per lane (coalesced index loads, no idle
// lanes waiting for long rows).  Each lane finds its entry's row (row_pos
// below), evaluates the pair, and a prefix sum over the batch's 64 lanes
// gives each row's part of the batch as the difference of the prefix values
// at the row's last and first lanes; the row's own lane adds that part to
// its accumulator.  The grid is persistent: each wave takes a contiguous
// range of 64-particle chunks, numbered XCD by XCD.

constexpr int kChunk = kWave;

// Chunks of this wave in the persistent grid.  Each XCD takes a contiguous
// share of the chunks (in proportion to its waves) and its waves take them
// interleaved (wave j of the XCD: j, j + W, j + 2W, ...), so at any moment
// an XCD's waves work on neighbouring chunks and the j-side gathers of one
// wave find the neighbourhood its siblings already brought into that XCD's
// L2.  Workgroups are dealt to the XCDs round-robin by their index.
struct ChunkWalk {
    int32_t first, end, stride;
};

__device__ __forceinline__ ChunkWalk chunk_walk(int32_t n_chunks)
{
    const int32_t groups = (int32_t)gridDim.x, p = (int32_t)blockIdx.x;
    const int32_t q = groups / 8, r = groups % 8;
    const int32_t xcd = p % 8, k = p / 8;
    const int32_t g0 = xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q;   // the XCD's first group
    const int32_t gx = q + (xcd < r ? 1 : 0);                                  // groups on the XCD
    const int32_t wpg = kBlock / kWave;
    const int64_t waves = (int64_t)groups * wpg;
    const int64_t w0 = (int64_t)g0 * wpg, wx = (int64_t)gx * wpg;
    ChunkWalk cw;
    // the wave's index is uniform across its lanes: say so, so that the
    // chunk, its particle range and (in a batch) its system are scalars
    cw.first = __builtin_amdgcn_readfirstlane((int32_t)(n_chunks * w0 / waves) + k * wpg +
                                              (int32_t)(threadIdx.x / kWave));
    cw.end = (int32_t)(n_chunks * (w0 + wx) / waves);
    cw.stride = (int32_t)wx;
    return cw;
}

// DPP lane moves (GFX9 data-parallel primitives): row_shr:d shifts inside
// each 16-lane row, row_bcast:15 / row_bcast:31 hand lane 15 of a row (lane
// 31) to the next row(s).  Lanes without a source read 0.
constexpr int kDppRowShr = 0x110;
constexpr int kDppBcast15 = 0x142;
constexpr int kDppBcast31 = 0x143;

template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, kRowMask, 0xF, false));
}

template <int kCtrl, int kRowMask>
__device__ __forceinline__ int32_t dpp_move(int32_t v)
{
    return __builtin_amdgcn_update_dpp(0, v, kCtrl, kRowMask, 0xF, false);
}

template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_move(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, kCtrl, kRowMask, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, kRowMask, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Inclusive prefix sum over all 64 lanes (no segments): shifts inside the
// 16-lane rows, then the row tails carried across rows.  Lanes without a
// source add 0, so no selects are needed.  A row of the batch is then the
// difference of two prefix values.
template <typename T>
__device__ __forceinline__ T wave_prefix(T v)
{
    v += dpp_move<kDppRowShr | 1, 0xF>(v);
    v += dpp_move<kDppRowShr | 2, 0xF>(v);
    v += dpp_move<kDppRowShr | 4, 0xF>(v);
    v += dpp_move<kDppRowShr | 8, 0xF>(v);
    v += dpp_move<kDppBcast15, 0xA>(v);
    v += dpp_move<kDppBcast31, 0xC>(v);
    return v;
}

// FP32 form: the two row-tail carries as single DPP adds (rows outside the
// row mask keep their value, the same result as adding the zero a masked
// move gives them).  The s_nops cover the wait a DPP read of a VGPR needs
// after a VALU write of it (before each add, and after the last for DPP
// reads the compiler places next, since it does not see into the asm).
template <>
__device__ __forceinline__ float wave_prefix<float>(float v)
{
    v += dpp_move<kDppRowShr | 1, 0xF>(v);
    v += dpp_move<kDppRowShr | 2, 0xF>(v);
    v += dpp_move<kDppRowShr | 4, 0xF>(v);
    v += dpp_move<kDppRowShr | 8, 0xF>(v);
    __asm__("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf" : "+v"(v));
    __asm__("s_nop 1\n\tv_add_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\ts_nop 1" : "+v"(v));
    return v;
}

// this row's part of batch [eb, eb+64) from the prefix values: lanes
// [first, last] (last = row_end_lane), zero when the row has no entry there
__device__ __forceinline__ float row_part(float prefix, int32_t first, int32_t last)
{
    const float hi = __shfl(prefix, last < 0 ? 0 : last, kWave);
    const float lo = __shfl(prefix, first > 0 ? first - 1 : 0, kWave);
    return last < 0 ? 0.f : (first > 0 ? hi - lo : hi);
}

__device__ __forceinline__ double row_part(double prefix, int32_t first, int32_t last)
{
    const double hi = __shfl(prefix, last < 0 ? 0 : last, kWave);
    const double lo = __shfl(prefix, first > 0 ? first - 1 : 0, kWave);
    return last < 0 ? 0.0 : (first > 0 ? hi - lo : hi);
}

// a slab entry's particle index and stencil code (-1: not coded)
__device__ __forceinline__ int32_t entry_j(int32_t raw, bool coded)
{
    return coded ? (raw & kSlabJMask) : raw;
}

__device__ __forceinline__ int32_t entry_code(int32_t raw, bool coded)
{
    return coded ? (int32_t)((uint32_t)raw >> kSlabCodeShift) : -1;
}

struct PairJob {
    const int32_t* cs;   // the chunk's first slab row (rows at cs[r * K], 32-bit offsets), or null
    int32_t i0, ni;      // first particle of the chunk, particles in it
    int32_t e0, e1;      // the entries walked (CSR positions, or with pairs
                         //   once the kept entries numbered from e0)
    int32_t rstart, rend;  // this lane's row among them (lane < ni)
    int32_t ni_once;     // pairs once: ni, or 0 when the chunk walks every entry
    int32_t sys;         // the chunk's system in a batch (one per chunk)
};

// The scalar parameters a pair reads, for a batch chunk's system: loaded
// once per chunk and made wave-uniform (scalar registers), where the pairs
// would otherwise read them from the batch table through vector loads.
struct PairParams {
    double L[3], halfL[3];
    double rc2, rl2, inv_rc, s, r_c;
    float cell_len32[3];
    int32_t nc[3];
    int32_t n_types;
    uint32_t seed_lo, seed_hi;
};

__device__ __forceinline__ double rfl(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)b);
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float rfl(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ int32_t rfl(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint32_t rfl(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

__device__ __forceinline__ PairParams pair_params(const KParams& K)
{
    PairParams p;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        p.L[d] = rfl(K.L[d]); p.halfL[d] = rfl(K.halfL[d]);
        p.cell_len32[d] = rfl(K.cell_len32[d]); p.nc[d] = rfl(K.nc[d]);
    }
    p.rc2 = rfl(K.rc2); p.rl2 = rfl(K.rl2); p.inv_rc = rfl(K.inv_rc); p.s = rfl(K.s); p.r_c = rfl(K.r_c);
    p.n_types = rfl(K.n_types);
    p.seed_lo = rfl(K.seed_lo); p.seed_hi = rfl(K.seed_hi);
    return p;
}

// A batch chunk's type tables (a, gamma, sigma / sqrt(dt)) copied into the
// wave's LDS rows: the chunk belongs to one system, so its pairs read the
// tables from LDS (and its scalar parameters from pair_params).
template <typename Tab>
__device__ __forceinline__ void stage_tables(const KParams& P, Tab* wa, Tab* wg, Tab* ws, int lane)
{
    const int nt2 = P.n_types * P.n_types;
    // the previous chunk's reads come first (one wave's LDS operations take
    // effect in program order)
    __asm__ __volatile__("" ::: "memory");
    for (int t = lane; t < nt2; t += kWave) {
        wa[t] = (Tab)P.a[t]; wg[t] = (Tab)P.g[t]; ws[t] = (Tab)P.srdt[t];
    }
    __asm__ __volatile__("" ::: "memory");
}

// Pairs once: per row of a wave's chunk (LDS, indexed by the wave's first
// thread + row), the row's first CSR entry and (entries below the chunk) |
// (mirror entries) << 16.
struct RowSkip {
    int32_t* raw;
    int32_t* skip;
};

constexpr int kPrePass = 16;    // row entries counted with independent loads

// chunk c: 64 rows from i0 (fewer at the end of the particle range).  In a
// batch, chunks are numbered system by system from each system's first
// particle, so every row is grouped, and its sum ordered, exactly as in the
// system's own single-system run.
//
// Pairs once (kSym): a pair of two particles of the same chunk is evaluated
// only from the lower row; its entry in the upper row (a "mirror") is left
// out of the walk and the lower row's evaluation adds the negated force to
// the upper particle through the wave's LDS accumulators.  Rows ascend, so a
// row's mirrors (chunk particles below it) are one run of entries after
// those below the chunk; the walk numbers the kept entries of the chunk's
// rows consecutively from e0 and maps them back to list positions.
template <bool kB, bool kSym>
__device__ __forceinline__ PairJob chunk_job(const BatchView& bv, const ForceArgs& a, const int32_t* slab,
                                             bool coded, const RowSkip& sk, int32_t c, bool ok, int lane)
{
    PairJob j;
    int32_t end = a.n;
    j.sys = 0;
    if constexpr (kB) {
        const int32_t sy = find_segment(bv.ch_off, bv.n_sys, c);
        j.sys = __builtin_amdgcn_readfirstlane(sy);
        j.i0 = bv.p_off[sy] + (c - bv.ch_off[sy]) * kChunk;
        end = bv.p_off[sy + 1];
    } else {
        j.i0 = c * kChunk;
    }
    j.ni = end - j.i0 < kChunk ? end - j.i0 : kChunk;
    j.cs = slab ? slab + (int64_t)j.i0 * a.slab_k : nullptr;
    const int32_t own = j.i0 + (lane < j.ni ? lane : j.ni - 1);
    j.e0 = ok ? a.offset[j.i0] : 0;
    j.e1 = ok ? a.offset[j.i0 + j.ni] : 0;
    j.rend = ok ? a.offset[own + 1] : 0;
    const int32_t prev = __shfl_up(j.rend, 1, kWave);
    j.rstart = lane == 0 ? j.e0 : prev;
    if (lane >= j.ni) { j.rstart = j.e1; j.rend = j.e1; }
    j.ni_once = 0;
    if constexpr (kSym) {
        const int32_t i = j.i0 + lane;
        const int32_t cnt = j.rend - j.rstart;
        int32_t below = 0, mir = 0;
        // count the row's entries below the chunk and below i: the first
        // kPrePass entries with independent loads, the rest (rows whose
        // mirrors reach further, rare) a group at a time; rows ascend
        for (int32_t p = 0; p < cnt; p += kPrePass) {
            int32_t jj[kPrePass];
#pragma unroll
            for (int q = 0; q < kPrePass; ++q) {
                const int32_t raw = p + q < cnt
                    ? (slab ? slab[(int64_t)i * a.slab_k + p + q] : a.index[j.rstart + p + q]) : 0x7fffffff;
                jj[q] = p + q < cnt ? entry_j(raw, coded) : 0x7fffffff;
            }
#pragma unroll
            for (int q = 0; q < kPrePass; ++q) {
                below += jj[q] < j.i0 ? 1 : 0;
                mir += (jj[q] >= j.i0 && jj[q] < i) ? 1 : 0;
            }
            if (jj[kPrePass - 1] > i) break;
        }
        // counts are packed in 16 bits: a chunk with a longer row walks
        // every entry (the choice covers both rows of each of its pairs)
        const bool once = !__any(cnt > 0xffff);
        if (!once) { below = 0; mir = 0; }
        j.ni_once = once ? j.ni : 0;
        const int32_t kept = cnt - mir;
        const int32_t incl = wave_prefix(kept);
        const int32_t tot = __shfl(incl, kWave - 1, kWave);
        // the previous chunk's reads of these slots come first (program
        // order of one wave's LDS operations)
        __asm__ __volatile__("" ::: "memory");
        sk.raw[lane] = j.rstart;
        sk.skip[lane] = below | (mir << 16);
        __asm__ __volatile__("" ::: "memory");
        j.rstart = j.e0 + incl - kept;
        j.rend = j.e0 + incl;
        j.e1 = j.e0 + tot;
    }
    return j;
}

// Row of this lane's entry e = eb + lane (the number of the chunk's rows
// that end at or before e), the lane where that row's part of the batch
// starts and the row's first entry.  Rows finished before the batch are
// counted with a ballot; each non-empty row starting inside the batch marks
// the lane of its first entry in a per-wave LDS row (LDS operations of one
// wave take effect in program order), and an inclusive prefix maximum over
// the lanes carries each mark to the row's later entries.
struct RowPos {
    int32_t r;
    int32_t start;       // first entry of the row (absolute)
};

// (marks are >= 0: an unsigned maximum, whose identity 0 lets the compiler
// fold each move into its DPP max)
__device__ __forceinline__ int32_t wave_max_prefix(int32_t v)
{
    uint32_t u = (uint32_t)v;
    u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, kDppRowShr | 1, 0xF, 0xF, false));
    u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, kDppRowShr | 2, 0xF, 0xF, false));
    u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, kDppRowShr | 4, 0xF, 0xF, false));
    u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, kDppRowShr | 8, 0xF, 0xF, false));
    u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, kDppBcast15, 0xA, 0xF, false));
    u = max(u, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)u, kDppBcast31, 0xC, 0xF, false));
    return (int32_t)u;
}

__device__ __forceinline__ RowPos row_pos(const PairJob& jb, int32_t eb, int lane, int32_t* __restrict__ s_mark)
{
    const bool own = lane < jb.ni;
    const int32_t ra = (int32_t)__popcll(__ballot(own && jb.rend <= eb));
    const int32_t p = jb.rstart - eb;
    // compiler memory barriers: the previous call's reads stay before these
    // writes, and the read below comes from LDS (other lanes' marks), never
    // from this lane's own store
    __asm__ __volatile__("" ::: "memory");
    s_mark[lane] = 0;
    if (own && jb.rend > jb.rstart && p >= 0 && p < kWave) s_mark[p] = lane + 1;
    __asm__ __volatile__("" ::: "memory");
    const int32_t v = wave_max_prefix(s_mark[lane]);
    int32_t r = (v > ra + 1 ? v : ra + 1) - 1;
    r = r < jb.ni ? r : jb.ni - 1;             // lanes past the last entry
    RowPos rp;
    rp.r = r;
    rp.start = __shfl(jb.rstart, r, kWave);
    return rp;
}

// Entry e of the chunk's rows: from the builder's fixed-width slab while it
// holds every row (row i at slab[i * K]), else from the CSR list.  With
// pairs once, e numbers the kept entries and skips the row's mirror run.
template <bool kSym>
__device__ __forceinline__ int32_t entry_at(const int32_t* __restrict__ slab, int32_t slab_k,
                                            const ForceArgs& a, const PairJob& jb, const RowPos& rp,
                                            const RowSkip& sk, int32_t e)
{
    // (slab rows through the chunk's base: a 32-bit offset per lane)
    if constexpr (kSym) {
        int32_t p = e - rp.start;
        const int32_t skip = sk.skip[rp.r];
        p += p >= (skip & 0xffff) ? (skip >> 16) : 0;
        if (slab) return jb.cs[rp.r * slab_k + p];
        return a.index[sk.raw[rp.r] + p];
    } else {
        return slab ? jb.cs[rp.r * slab_k + (e - rp.start)] : a.index[e];
    }
}

// the slab when it is usable for this launch, else null
__device__ __forceinline__ const int32_t* usable_slab(const ForceArgs& a)
{
    return (a.slab && *a.slab_flag == 0) ? a.slab : nullptr;
}

// lane holding the last entry of this lane's row inside batch [eb, eb+64),
// or -1 when the row has no entry there
__device__ __forceinline__ int32_t row_end_lane(const PairJob& jb, int32_t eb)
{
    const int32_t lo = jb.rstart > eb ? jb.rstart : eb;
    int32_t hi = jb.rend < eb + kWave ? jb.rend : eb + kWave;
    return lo < hi ? hi - eb - 1 : -1;
}

// One pair (FP64): force contribution on i and its half of the pair
// potential.  P supplies geometry and cutoff; A / G / S the type tables
// (a, gamma, sigma / sqrt(dt)).
// One particle's operands of the FP64 pair: from the packed copies when
// the step wrote them, else from the state's arrays.
struct Op64 {
    double x, y, z, vx, vy, vz;
    uint32_t tag;
    int32_t type;
};

// The packed FP64 records through buffer resources (32-bit byte offsets,
// n < 2^26), as two 16-byte loads each.
struct Src64 {
    __amdgpu_buffer_rsrc_t x, v;
};

__device__ __forceinline__ Src64 src64(const ForceArgs& a)
{
    const int32_t bytes = a.x64 && a.n < (1 << 26) ? a.n * (int32_t)sizeof(double4) : 0;
    return Src64{__builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(a.x64), (short)0, bytes, 0x00020000),
                 __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(a.v64), (short)0, bytes, 0x00020000)};
}

__device__ __forceinline__ double4 rec64(__amdgpu_buffer_rsrc_t r, int32_t k)
{
    const int32_t o = k * (int32_t)sizeof(double4);
    const auto lo = __builtin_amdgcn_raw_buffer_load_b128(r, o, 0, 0);
    const auto hi = __builtin_amdgcn_raw_buffer_load_b128(r, o + 16, 0, 0);
    auto d = [](int a, int b) { return __longlong_as_double(((long long)(uint32_t)b << 32) | (uint32_t)a); };
    double4 r4;
    r4.x = d(lo[0], lo[1]); r4.y = d(lo[2], lo[3]); r4.z = d(hi[0], hi[1]); r4.w = d(hi[2], hi[3]);
    return r4;
}

__device__ __forceinline__ Op64 load_op64(const ForceArgs& a, const Src64& sr, int64_t N, int32_t i)
{
    Op64 o;
    if (a.x64) {
        double4 p, q;
        if (a.n < (1 << 26)) {
            p = rec64(sr.x, i);
            q = rec64(sr.v, i);
        } else {
            p = reinterpret_cast<const double4*>(a.x64)[i];
            q = reinterpret_cast<const double4*>(a.v64)[i];
        }
        o.x = p.x; o.y = p.y; o.z = p.z;
        o.vx = q.x; o.vy = q.y; o.vz = q.z;
        o.tag = (uint32_t)__double_as_longlong(p.w);
        o.type = (int32_t)__double_as_longlong(q.w);
    } else {
        o.x = a.x[i]; o.y = a.x[N + i]; o.z = a.x[2 * N + i];
        o.vx = a.v[i]; o.vy = a.v[N + i]; o.vz = a.v[2 * N + i];
        o.tag = a.tag[i];
        o.type = a.type[i];
    }
    return o;
}

// A wave-uniform seed is passed through an empty asm statement before each
// pair's hash: the compiler then forms the ten round keys with scalar adds
// at the point of use instead of keeping twenty of them live across the
// loop (which overflows the scalar registers into lane spills).
template <bool kUniform>
__device__ __forceinline__ void opaque_keys(uint32_t& s0, uint32_t& s1)
{
    if constexpr (kUniform) __asm__ volatile("" : "+s"(s0), "+s"(s1));
}

template <int kWMode, bool kUniform, typename PT>
__device__ __forceinline__ bool pair64(const PT& P, const double* A, const double* G, const double* S,
                                       const Op64& oi, const Op64& oj, uint64_t step,
                                       double& px, double& py, double& pz, double& pp)
{
    const double dx = min_image(oi.x - oj.x, P.L[0], P.halfL[0]);
    const double dy = min_image(oi.y - oj.y, P.L[1], P.halfL[1]);
    const double dz = min_image(oi.z - oj.z, P.L[2], P.halfL[2]);
    const double r2 = dist2(dx, dy, dz);
    if (!(r2 < P.rc2)) return false;
    const double rr = sqrt(r2);
    // one correctly rounded reciprocal for the three components (within an
    // ulp of the three quotients)
    const double inv_r = 1.0 / rr;
    const double ex = dx * inv_r, ey = dy * inv_r, ez = dz * inv_r;
    const double wc = 1.0 - rr * P.inv_rc;
    const double wr = weight_r(wc, kWMode, P.s);
    const double wd = wr * wr;
    const double ev = ex * (oi.vx - oj.vx) + ey * (oi.vy - oj.vy) + ez * (oi.vz - oj.vz);
    const int tp = oi.type * P.n_types + oj.type;
    uint32_t s0 = P.seed_lo, s1 = P.seed_hi;
    opaque_keys<kUniform>(s0, s1);
    const double xi_ij = gauss64(pair_words(oi.tag, oj.tag, step, s0, s1));
    const double phi = A[tp] * wc - G[tp] * wd * ev + S[tp] * wr * xi_ij;
    px = phi * ex; py = phi * ey; pz = phi * ez;
    pp = 0.25 * A[tp] * P.r_c * wc * wc;
    return true;
}

template <int kWMode, bool kB, bool kSym, bool kVV = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_force_fp64(KParams kp, BatchView bv, ForceArgs a, int32_t n_chunks)
{
    __shared__ double s_a[kTab], s_g[kTab], s_s[kTab];
    // kVV (single systems): the step's half-kicks in the row epilogue, with
    // their momentum and |v|^2 accumulators per lane
    static_assert(!(kVV && kB), "the fused half-kick is for single systems");
    __shared__ double s_vacc[kVV ? 6 * kBlock : 1];
    if constexpr (kVV) {
        for (int k = 0; k < 6; ++k) s_vacc[k * kBlock + threadIdx.x] = 0.0;
    }
    __shared__ int32_t s_rowm[kBlock];                 // per-wave row marks (row_pos)
    // pairs once: the mirrored contributions to the wave's 64 rows
    __shared__ double s_jx[kSym ? kBlock : 1], s_jy[kSym ? kBlock : 1], s_jz[kSym ? kBlock : 1];
    __shared__ double s_jp[kSym ? kBlock : 1];
    __shared__ int32_t s_jn[kSym ? kBlock : 1];
    __shared__ int32_t s_raw[kSym ? kBlock : 1], s_skip[kSym ? kBlock : 1];
    // a batch: each wave's own copy of its chunk's tables
    __shared__ double s_wt[kB ? 3 * (kBlock / kWave) * kTab : 1];
    if (!kB) {
        const int nt2 = kp.n_types * kp.n_types;
        for (int t = threadIdx.x; t < nt2; t += kBlock) {
            s_a[t] = kp.a[t]; s_g[t] = kp.g[t]; s_s[t] = kp.srdt[t];
        }
        __syncthreads();
    }
    double* const wt = s_wt + (kB ? 3 * kTab * (int)(threadIdx.x / kWave) : 0);
    const int lane = threadIdx.x & (kWave - 1);
    int32_t* const s_mark = s_rowm + (threadIdx.x - lane);
    const int wbase = threadIdx.x - lane;
    const int sb = kSym ? wbase : 0;
    const RowSkip sk{s_raw + sb, s_skip + sb};
    if constexpr (kSym) {
        s_jx[threadIdx.x] = 0.0; s_jy[threadIdx.x] = 0.0; s_jz[threadIdx.x] = 0.0;
        s_jp[threadIdx.x] = 0.0; s_jn[threadIdx.x] = 0;
    }
    const ChunkWalk cw = chunk_walk(n_chunks);
    const int64_t N = a.n;
    const uint64_t step = (a.d_step ? *a.d_step : 0ull) + a.step_add;
    const bool ok = (int64_t)a.offset[a.n] <= a.capacity;
    const bool want_pe = a.pe != nullptr;
    const bool want_np = a.npair != nullptr;
    double pe_tot = 0.0, np_tot = 0.0;
    const int32_t* __restrict__ slab = usable_slab(a);
    const bool coded = slab && a.slab_coded;
    const Src64 sr = src64(a);
    for (int32_t c = cw.first; c < cw.end; c += cw.stride) {
        const PairJob jb = chunk_job<kB, kSym>(bv, a, slab, coded, sk, c, ok, lane);
        PairParams pp_sys;
        if constexpr (kB) {
            stage_tables(bv.kps[jb.sys], wt, wt + kTab, wt + 2 * kTab, lane);
            pp_sys = pair_params(bv.kps[jb.sys]);
        }
        double fx = 0.0, fy = 0.0, fz = 0.0, pe_row = 0.0, np_row = 0.0;
        // the list entries are requested a batch ahead of their use
        RowPos rp_nxt = row_pos(jb, jb.e0, lane, s_mark);
        int32_t raw_nxt = jb.e0 + lane < jb.e1 ? entry_at<kSym>(slab, a.slab_k, a, jb, rp_nxt, sk, jb.e0 + lane) : 0;
        for (int32_t eb = jb.e0; eb < jb.e1; eb += kWave) {
            const int32_t e = eb + lane;
            const bool valid = e < jb.e1;
            const RowPos rp = rp_nxt;
            const int32_t raw = raw_nxt;
            // (unguarded: a request past the chunk's last entry is masked
            // off per lane, and no register copy at a join waits for it)
            rp_nxt = row_pos(jb, eb + kWave, lane, s_mark);
            raw_nxt = e + kWave < jb.e1 ? entry_at<kSym>(slab, a.slab_k, a, jb, rp_nxt, sk, e + kWave) : 0;
            const int32_t r = rp.r;
            const int32_t i = jb.i0 + r;
            const int32_t j = valid ? entry_j(raw, coded) : i;
            double px = 0.0, py = 0.0, pz = 0.0, pp = 0.0, pn = 0.0;
            if (valid) {
                bool hit;
                if constexpr (kB) {
                    hit = pair64<kWMode, true>(pp_sys, wt, wt + kTab, wt + 2 * kTab, load_op64(a, sr, N, i),
                                               load_op64(a, sr, N, j), step, px, py, pz, pp);
                } else {
                    hit = pair64<kWMode, true>(kp, s_a, s_g, s_s, load_op64(a, sr, N, i), load_op64(a, sr, N, j),
                                               step, px, py, pz, pp);
                }
                pn = hit ? 1.0 : 0.0;
                np_tot += pn;
                if constexpr (kSym) {
                    // a pair inside the chunk: the upper particle's share
                    if (hit && (uint32_t)(j - jb.i0) < (uint32_t)jb.ni_once) {
                        const int q = wbase + (j - jb.i0);
                        atomicAdd(&s_jx[q], -px);
                        atomicAdd(&s_jy[q], -py);
                        atomicAdd(&s_jz[q], -pz);
                        if (want_pe) atomicAdd(&s_jp[q], pp);
                        if (want_np) atomicAdd(&s_jn[q], 1);
                        np_tot += 1.0;
                        pe_tot += pp;
                    }
                }
            }
            pe_tot += pp;
            // each row's part of the batch as the difference of two prefix
            // sums over the batch (the prefix values stay within a few
            // hundred, so a part carries an error of a few ulp of that,
            // far below the per-particle bar)
            px = wave_prefix(px);
            py = wave_prefix(py);
            pz = wave_prefix(pz);
            if (want_pe) pp = wave_prefix(pp);
            if (want_np) pn = wave_prefix(pn);
            const int32_t src = row_end_lane(jb, eb);
            const int32_t first = jb.rstart - eb;
            const double tx = row_part(px, first, src);
            const double ty = row_part(py, first, src);
            const double tz = row_part(pz, first, src);
            const double tp2 = want_pe ? row_part(pp, first, src) : 0.0;
            const double tn = want_np ? row_part(pn, first, src) : 0.0;
            if (src >= 0) { fx += tx; fy += ty; fz += tz; pe_row += tp2; np_row += tn; }
        }
        if constexpr (kSym) {
            // LDS operations of one wave take effect in program order
            __asm__ __volatile__("" ::: "memory");
            fx += s_jx[threadIdx.x]; fy += s_jy[threadIdx.x]; fz += s_jz[threadIdx.x];
            pe_row += s_jp[threadIdx.x]; np_row += (double)s_jn[threadIdx.x];
            s_jx[threadIdx.x] = 0.0; s_jy[threadIdx.x] = 0.0; s_jz[threadIdx.x] = 0.0;
            s_jp[threadIdx.x] = 0.0; s_jn[threadIdx.x] = 0;
            __asm__ __volatile__("" ::: "memory");
        }
        if (lane < jb.ni) {
            const int32_t i = jb.i0 + lane;
            double pe_b = 0.0;
            if constexpr (kB) add_bonds_body(bv.kps[jb.sys], a, i, a.x[i], a.x[N + i], a.x[2 * N + i], fx, fy, fz, pe_b);
            else add_bonds_body(kp, a, i, a.x[i], a.x[N + i], a.x[2 * N + i], fx, fy, fz, pe_b);
            pe_tot += pe_b;
            a.f[i] = fx;
            a.f[N + i] = fy;
            a.f[2 * N + i] = fz;
            if (want_pe) a.pe[i] = pe_row + pe_b;
            if (want_np) a.npair[i] = (int32_t)np_row;
            if constexpr (kVV) {
                // (the operands are requested here, not held through the
                // chunk: the pass has no registers to spare; other waves
                // cover the wait)
                const VVIn vin = vv_load(a, N, i);
                vv_row(kp, a, N, i, vin, fx, fy, fz, s_vacc + threadIdx.x);
            }
        }
    }
    if (a.fred_part) block_partials2(pe_tot, 0.5 * np_tot, a.fred_part);
    if constexpr (kVV) vv_partials(s_vacc, a.vv_part);
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

// The operands of one mixed-form pair, loaded a batch ahead of their use:
// xw[i] = (x, y, z offsets inside the cell, tag bits), vw[i] = (predicted
// velocity, type), both float4; the packed cells are read only for list
// entries without a stencil code.
struct PairIn {
    float4 pi, qi, pj, qj;
    uint32_t ci, cj;
};

// The packed records through buffer resources: 32-bit byte offsets (n <
// 2^28) instead of 64-bit addresses per gather, and a record past the end
// reads zero instead of faulting.
struct MixedSrc {
    __amdgpu_buffer_rsrc_t xw, vw;
};

__device__ __forceinline__ MixedSrc mixed_src(const ForceArgs& a)
{
    const int32_t bytes = a.n * (int32_t)sizeof(float4);
    return MixedSrc{__builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.x32), (short)0, bytes, 0x00020000),
                    __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.v32), (short)0, bytes, 0x00020000)};
}

__device__ __forceinline__ float4 rec4(__amdgpu_buffer_rsrc_t r, int32_t k)
{
    const auto w = __builtin_amdgcn_raw_buffer_load_b128(r, k * (int32_t)sizeof(float4), 0, 0);
    return make_float4(__int_as_float(w[0]), __int_as_float(w[1]), __int_as_float(w[2]), __int_as_float(w[3]));
}

__device__ __forceinline__ PairIn load_pair(const ForceArgs& a, const MixedSrc& src, int32_t i, int32_t j,
                                            bool coded)
{
    PairIn in;
    in.pi = rec4(src.xw, i); in.qi = rec4(src.vw, i);
    in.pj = rec4(src.xw, j); in.qj = rec4(src.vw, j);
    in.ci = 0u; in.cj = 0u;
    if (!coded) { in.ci = a.cell_xyz[i]; in.cj = a.cell_xyz[j]; }
    return in;
}

// one batch's row position, pair and operands in the mixed pipeline
struct Stage {
    RowPos rp;
    int32_t i, j, code;
    PairIn in;
};

template <int kWMode, bool kUniform, typename PT, typename Tab>
__device__ __forceinline__ bool pair32(const PT& P, const Tab* A, const Tab* G, const Tab* S,
                                       const float4* __restrict__ offs, bool skin, const ForceArgs& a,
                                       const PairIn& in, int64_t N, int32_t i, int32_t j, int32_t code,
                                       bool coded, bool valid, uint64_t step, float& px, float& py, float& pz,
                                       float& pp)
{
    const float4 pi = in.pi, qi = in.qi;
    const float4 pj = in.pj, qj = in.qj;
    // whole-cell offset of i's cell from j's: from the list entry's stencil
    // code when it has one (a table of the 27 offsets in the wave's LDS),
    // else from the two cells' coordinates
    float ox, oy, oz;
    if (coded) {
        const float4 o = offs[code];
        ox = o.x; oy = o.y; oz = o.z;
    } else {
        const uint32_t ci = in.ci, cj = in.cj;
        ox = (float)cell_delta((int32_t)(ci & 1023u), (int32_t)(cj & 1023u), P.nc[0]) * P.cell_len32[0];
        oy = (float)cell_delta((int32_t)((ci >> 10) & 1023u), (int32_t)((cj >> 10) & 1023u), P.nc[1]) * P.cell_len32[1];
        oz = (float)cell_delta((int32_t)(ci >> 20), (int32_t)(cj >> 20), P.nc[2]) * P.cell_len32[2];
    }
    const float dx = (pi.x - pj.x) + ox;
    const float dy = (pi.y - pj.y) + oy;
    const float dz = (pi.z - pj.z) + oz;
    const float r2 = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
    // with no skin the FP64 list already decided the pair set; a skin needs
    // the FP32 test (documented reading).  Lanes without a pair (past the
    // batch's end) run the same arithmetic on their own particle and are
    // zeroed at the end, so the common path has no branches.
    bool hit = valid;
    if (skin) hit = hit && r2 < (float)P.rc2;
    const float inv_r = __builtin_amdgcn_rsqf(r2);
    float rr = r2 * inv_r;
    float ex = dx * inv_r, ey = dy * inv_r, ez = dz * inv_r;
    if (hit && r2 < kCloseR2) {
        // FP32 offsets cannot resolve the direction of a nearly coincident
        // pair: take its geometry from FP64 positions
        const double ddx = min_image(a.x[i] - a.x[j], P.L[0], P.halfL[0]);
        const double ddy = min_image(a.x[N + i] - a.x[N + j], P.L[1], P.halfL[1]);
        const double ddz = min_image(a.x[2 * N + i] - a.x[2 * N + j], P.L[2], P.halfL[2]);
        const double r64 = sqrt(dist2(ddx, ddy, ddz));
        if (r64 > 0.0) {
            rr = (float)r64;
            ex = (float)(ddx / r64); ey = (float)(ddy / r64); ez = (float)(ddz / r64);
        } else {
            hit = false;                               // coincident: no direction, no force
        }
    }
    float wc = __fmaf_rn(-rr, (float)P.inv_rc, 1.0f);
    wc = wc > 0.f ? wc : 0.f;
    const float wr = weight_r32(wc, kWMode, (float)P.s);
    const float wd = kWMode == 0 ? wc : wr * wr;     // s = 1/2: w_D = w_R^2 = w_C exactly
    const float ev = __fmaf_rn(ez, qi.z - qj.z, __fmaf_rn(ey, qi.y - qj.y, ex * (qi.x - qj.x)));
    const int tp = (int)__float_as_uint(qi.w) * P.n_types + (int)__float_as_uint(qj.w);
    uint32_t s0 = P.seed_lo, s1 = P.seed_hi;
    opaque_keys<kUniform>(s0, s1);
    const float xi_ij = gauss32(pair_words(__float_as_uint(pi.w), __float_as_uint(pj.w), step, s0, s1));
    const float at = (float)A[tp], gt = (float)G[tp], st = (float)S[tp];
    const float phi = __fmaf_rn(at, wc, __fmaf_rn(-(gt * wd), ev, (st * wr) * xi_ij));
    px = hit ? phi * ex : 0.f;
    py = hit ? phi * ey : 0.f;
    pz = hit ? phi * ez : 0.f;
    pp = hit ? 0.25f * (float)P.r_c * at * wc * wc : 0.f;
    return hit;
}

// One particle's operands of the filter's distance test: its FP32
// cell-relative position and cell word (mixed form; the word only when list
// entries carry no stencil code), or its FP64 position (FP64 form).
template <bool kMixed> struct SkinOp;
template <> struct SkinOp<true> {
    float x, y, z;
    uint32_t cell;
};
template <> struct SkinOp<false> {
    double x, y, z;
};

template <bool kMixed>
__device__ __forceinline__ SkinOp<kMixed> skin_op(const ForceArgs& a, int32_t k, bool coded)
{
    SkinOp<kMixed> o;
    if constexpr (kMixed) {
        const float4 p = rec4(mixed_src(a).xw, k);
        o.x = p.x; o.y = p.y; o.z = p.z;
        o.cell = coded ? 0u : a.cell_xyz[k];
    } else {
        const Op64 q = load_op64(a, src64(a), a.n, k);
        o.x = q.x; o.y = q.y; o.z = q.z;
    }
    return o;
}

// the operands that lane src holds
template <bool kMixed>
__device__ __forceinline__ SkinOp<kMixed> skin_op_of(const SkinOp<kMixed>& own, int src, bool coded)
{
    SkinOp<kMixed> o;
    o.x = __shfl(own.x, src, kWave);
    o.y = __shfl(own.y, src, kWave);
    o.z = __shfl(own.z, src, kWave);
    if constexpr (kMixed) o.cell = coded ? 0u : (uint32_t)__shfl((int32_t)own.cell, src, kWave);
    return o;
}

// r < r_c for one entry, on the arithmetic of the form's force pass
// (offs: the whole-cell offsets of the 64 stencil codes, as the force pass
// stages them)
template <bool kMixed>
__device__ __forceinline__ bool skin_hit(const KParams& kp, const float4* __restrict__ offs,
                                         const SkinOp<kMixed>& pi, const SkinOp<kMixed>& pj, int32_t code, bool coded)
{
    if constexpr (kMixed) {
        float ox, oy, oz;
        if (coded) {
            const float4 o = offs[code];
            ox = o.x; oy = o.y; oz = o.z;
        } else {
            const uint32_t ci = pi.cell, cj = pj.cell;
            ox = (float)cell_delta((int32_t)(ci & 1023u), (int32_t)(cj & 1023u), kp.nc[0]) * kp.cell_len32[0];
            oy = (float)cell_delta((int32_t)((ci >> 10) & 1023u), (int32_t)((cj >> 10) & 1023u), kp.nc[1]) *
                 kp.cell_len32[1];
            oz = (float)cell_delta((int32_t)(ci >> 20), (int32_t)(cj >> 20), kp.nc[2]) * kp.cell_len32[2];
        }
        const float dx = (pi.x - pj.x) + ox;
        const float dy = (pi.y - pj.y) + oy;
        const float dz = (pi.z - pj.z) + oz;
        return __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx)) < (float)kp.rc2;
    } else {
        const double dx = min_image(pi.x - pj.x, kp.L[0], kp.halfL[0]);
        const double dy = min_image(pi.y - pj.y, kp.L[1], kp.halfL[1]);
        const double dz = min_image(pi.z - pj.z, kp.L[2], kp.halfL[2]);
        return dist2(dx, dy, dz) < kp.rc2;
    }
}

constexpr int kSkinGroup = 4;    // batches of the filter whose loads are in flight together

// Rows of the pairs inside r_c out of a list built at r_c + skin, for the
// force pass of every step (those between rebuilds keep the last build's
// rows while the particles move).  A wave takes 64 rows and walks their
// entries 64 at a time, as the force pass does: each lane tests its entry's
// current separation, a ballot gives the batch's hits, and a hit goes to
// its row's next free slot of the kept rows (same slab layout): the row's
// count so far plus the hits on the row's lower lanes of the batch (mbcnt).
// count[i] gets each row's kept number (scanned into offsets afterwards).
// The mixed form decides on the FP32 separation its force pass computes
// (in-cell offsets plus the whole-cell offset of the entry's stencil code,
// or of the two cells when entries are not coded), the FP64 form on the
// FP64 rule.  Each row's own operands come once per chunk, from its lane;
// the partners' loads of kSkinGroup batches are issued together, with the
// list entries of the next group behind them, so a wave waits once per
// group rather than once per batch.  (A lane per row instead spreads every
// load over 64 rows' cache lines, and ran 2.6 times slower.)
//
// When the builder's slab did not hold every row (its rows then come from
// the CSR list, and a kept row might not fit a slab row), the rows pass
// unfiltered: count[i] gets the CSR row size and *kept_flag = 1 makes the
// force pass read the CSR list (whose offsets the scanned counts then are)
// and test r < r_c itself.
template <bool kMixed, bool kCoded>
__global__ __launch_bounds__(kBlock) void k_skin_filter(KParams kp, ForceArgs a, int32_t* __restrict__ kept,
                                                        int32_t* __restrict__ count, int32_t* __restrict__ kept_flag)
{
    __shared__ int32_t s_rowm[kBlock];
    __shared__ float4 s_off[kWave];
    const int lane = threadIdx.x & (kWave - 1);
    int32_t* const s_mark = s_rowm + (threadIdx.x - lane);
    const bool ok = (int64_t)a.offset[a.n] <= a.capacity;
    const int32_t* __restrict__ slab = usable_slab(a);
    if (!slab) {
        for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < a.n; i += gridDim.x * kBlock)
            count[i] = ok ? a.offset[i + 1] - a.offset[i] : 0;
        if (blockIdx.x == 0 && threadIdx.x == 0) *kept_flag = 1;
        return;
    }
    if (threadIdx.x < kWave) {
        const int t = threadIdx.x;
        s_off[t] = make_float4((float)(1 - (t & 3)) * kp.cell_len32[0], (float)(1 - ((t >> 2) & 3)) * kp.cell_len32[1],
                               (float)(1 - (t >> 4)) * kp.cell_len32[2], 0.f);
    }
    __syncthreads();
    const int32_t K = a.slab_k;
    const int32_t n_chunks = (a.n + kChunk - 1) / kChunk;
    const int32_t waves = (int32_t)gridDim.x * (kBlock / kWave);
    const int32_t w0 = __builtin_amdgcn_readfirstlane((int32_t)blockIdx.x * (kBlock / kWave) +
                                                      (int32_t)(threadIdx.x / kWave));
    const BatchView none{};
    const RowSkip sk{nullptr, nullptr};
    for (int32_t c = w0; c < n_chunks; c += waves) {
        const PairJob jb = chunk_job<false, false>(none, a, slab, kCoded, sk, c, ok, lane);
        const SkinOp<kMixed> own = skin_op<kMixed>(a, jb.i0 + (lane < jb.ni ? lane : jb.ni - 1), kCoded);
        // the chunk's rows of the slab and of the kept rows, addressed from
        // their first row with 32-bit offsets (64 rows of K entries)
        const int32_t* __restrict__ cs = slab + (int64_t)jb.i0 * K;
        int32_t* __restrict__ ck = kept + (int64_t)jb.i0 * K;
        // a row's entry of batch eb for this lane (its own particle past the end)
        auto entry = [&](const RowPos& rp, int32_t eb) {
            const int32_t e = eb + lane;
            return e < jb.e1 ? cs[rp.r * K + (e - rp.start)] : jb.i0 + rp.r;
        };
        RowPos rp_n[kSkinGroup];
        int32_t raw_n[kSkinGroup];
#pragma unroll
        for (int q = 0; q < kSkinGroup; ++q) {
            rp_n[q] = row_pos(jb, jb.e0 + q * kWave, lane, s_mark);
            raw_n[q] = entry(rp_n[q], jb.e0 + q * kWave);
        }
        int32_t kc = 0;                            // this lane's row (lane < ni): entries kept so far
        for (int32_t eg = jb.e0; eg < jb.e1; eg += kSkinGroup * kWave) {
            RowPos rp[kSkinGroup];
            int32_t raw[kSkinGroup];
            SkinOp<kMixed> pj[kSkinGroup];
#pragma unroll
            for (int q = 0; q < kSkinGroup; ++q) {
                rp[q] = rp_n[q];
                raw[q] = raw_n[q];
                pj[q] = skin_op<kMixed>(a, entry_j(raw[q], kCoded), kCoded);
            }
#pragma unroll
            for (int q = 0; q < kSkinGroup; ++q) {
                const int32_t e = eg + (kSkinGroup + q) * kWave;
                rp_n[q] = row_pos(jb, e, lane, s_mark);
                raw_n[q] = entry(rp_n[q], e);
            }
#pragma unroll
            for (int q = 0; q < kSkinGroup; ++q) {
                const int32_t eb = eg + q * kWave;
                const SkinOp<kMixed> pi = skin_op_of<kMixed>(own, rp[q].r, kCoded);
                const bool hit =
                    eb + lane < jb.e1 && skin_hit<kMixed>(kp, s_off, pi, pj[q], entry_code(raw[q], kCoded), kCoded);
                const uint64_t hb = __ballot(hit);
                const int32_t below = lanes_below(hb);            // hits on lower lanes of the batch
                const int32_t first = rp[q].start - eb > 0 ? rp[q].start - eb : 0;
                const int32_t below_first = __shfl(below, first & (kWave - 1), kWave);
                const int32_t base = __shfl(kc, rp[q].r, kWave);   // the row's kept entries before the batch
                if (hit) ck[rp[q].r * K + base + (below - below_first)] = raw[q];
                // each row's own lane adds the row's hits in this batch
                const int32_t last = row_end_lane(jb, eb);
                const int32_t my_first = jb.rstart - eb > 0 ? jb.rstart - eb : 0;
                const int32_t upto = __shfl(below + (hit ? 1 : 0), last < 0 ? 0 : last, kWave);
                const int32_t from = __shfl(below, my_first & (kWave - 1), kWave);
                if (last >= 0) kc += upto - from;
            }
        }
        if (lane < jb.ni) count[jb.i0 + lane] = kc;
    }
}

// Mixed form.  Pair terms in FP32, the batch prefix sums in FP32, each row's
// batch parts added with a two-sum, the result stored in FP64.
template <int kWMode, bool kB, bool kSym, bool kVV>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_force_mixed(KParams kp, BatchView bv, ForceArgs a, int32_t n_chunks)
{
    __shared__ float s_a[kTab], s_g[kTab], s_s[kTab];
    __shared__ int32_t s_rowm[kBlock];                 // per-wave row marks (row_pos)
    // pairs once: the mirrored contributions to the wave's 64 rows
    __shared__ float s_jx[kSym ? kBlock : 1], s_jy[kSym ? kBlock : 1], s_jz[kSym ? kBlock : 1];
    __shared__ float s_jp[kSym ? kBlock : 1];
    __shared__ int32_t s_jn[kSym ? kBlock : 1];
    __shared__ int32_t s_raw[kSym ? kBlock : 1], s_skip[kSym ? kBlock : 1];
    // a batch: each wave's own copy of its chunk's tables
    __shared__ float s_wt[kB ? 3 * (kBlock / kWave) * kTab : 1];
    // each wave's table of the whole-cell offsets of the 64 stencil codes
    // (ex | ey << 2 | ez << 4 -> ((1 - ex) l_x, (1 - ey) l_y, (1 - ez) l_z),
    // the cell lengths of the wave's system)
    __shared__ float4 s_off[(kBlock / kWave) * kWave];
    // kVV (single systems): the step's half-kicks in the row epilogue, with
    // their momentum and |v|^2 accumulators per lane
    static_assert(!(kVV && kB), "the fused half-kick is for single systems");
    constexpr bool vv = kVV;
    __shared__ double s_vacc[kVV ? 6 * kBlock : 1];
    if constexpr (kVV) {
        for (int k = 0; k < 6; ++k) s_vacc[k * kBlock + threadIdx.x] = 0.0;
    }
    const int lane = threadIdx.x & (kWave - 1);
    float4* const offs = s_off + (threadIdx.x - lane);
    auto stage_offsets = [&](const KParams& P) {
        __asm__ __volatile__("" ::: "memory");
        offs[lane] = make_float4((float)(1 - (lane & 3)) * P.cell_len32[0],
                                 (float)(1 - ((lane >> 2) & 3)) * P.cell_len32[1],
                                 (float)(1 - (lane >> 4)) * P.cell_len32[2], 0.f);
        __asm__ __volatile__("" ::: "memory");
    };
    if (!kB) {
        const int nt2 = kp.n_types * kp.n_types;
        for (int t = threadIdx.x; t < nt2; t += kBlock) {
            s_a[t] = (float)kp.a[t]; s_g[t] = (float)kp.g[t]; s_s[t] = (float)kp.srdt[t];
        }
        stage_offsets(kp);
        __syncthreads();
    }
    // lists built with a skin: the FP32 separation decides r < r_c
    bool skin = __builtin_amdgcn_readfirstlane(kp.rl2 != kp.rc2 ? 1 : 0) != 0;
    float* const wt = s_wt + (kB ? 3 * kTab * (int)(threadIdx.x / kWave) : 0);
    int32_t* const s_mark = s_rowm + (threadIdx.x - lane);
    const int wbase = threadIdx.x - lane;
    const int sb = kSym ? wbase : 0;
    const RowSkip sk{s_raw + sb, s_skip + sb};
    if constexpr (kSym) {
        s_jx[threadIdx.x] = 0.f; s_jy[threadIdx.x] = 0.f; s_jz[threadIdx.x] = 0.f;
        s_jp[threadIdx.x] = 0.f; s_jn[threadIdx.x] = 0;
    }
    const ChunkWalk cw = chunk_walk(n_chunks);
    const int64_t N = a.n;
    const uint64_t step = (a.d_step ? *a.d_step : 0ull) + a.step_add;
    const bool ok = (int64_t)a.offset[a.n] <= a.capacity;
    const bool want_pe = a.pe != nullptr;
    const bool want_np = a.npair != nullptr;
    const MixedSrc src = mixed_src(a);
    const int32_t* __restrict__ slab = usable_slab(a);
    const bool coded = slab && a.slab_coded;
    double pe_tot = 0.0;
    int32_t np_tot = 0;                        // pairs inside r_c seen by this lane
    for (int32_t c = cw.first; c < cw.end; c += cw.stride) {
        const PairJob jb = chunk_job<kB, kSym>(bv, a, slab, coded, sk, c, ok, lane);
        PairParams pp_sys;
        if constexpr (kB) {
            stage_tables(bv.kps[jb.sys], wt, wt + kTab, wt + 2 * kTab, lane);
            stage_offsets(bv.kps[jb.sys]);
            pp_sys = pair_params(bv.kps[jb.sys]);
            skin = pp_sys.rl2 != pp_sys.rc2;
        }
        float sx = 0.f, sy = 0.f, sz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f, pe_row = 0.f, np_row = 0.f;
        // the half-kick's operands of this lane's row, requested now
        VVIn vin{};
        if constexpr (kVV) {
            if (lane < jb.ni) vin = vv_load(a, N, jb.i0 + lane);
        }
        // software pipeline: the list entry two batches ahead and the pair
        // operands one batch ahead are requested before a batch is evaluated;
        // two stages alternate (the loop is unrolled by two) so no operand is
        // copied from one to the other
        Stage A, B;
        A.rp = row_pos(jb, jb.e0, lane, s_mark);
        A.i = jb.i0 + A.rp.r;
        const int32_t raw0 = jb.e0 + lane < jb.e1 ? entry_at<kSym>(slab, a.slab_k, a, jb, A.rp, sk, jb.e0 + lane) : A.i;
        A.j = entry_j(raw0, coded);
        A.code = entry_code(raw0, coded);
        A.in = load_pair(a, src, A.i, A.j, coded);
        RowPos rp_nxt = row_pos(jb, jb.e0 + kWave, lane, s_mark);
        int32_t raw_nxt = jb.e0 + kWave + lane < jb.e1
            ? entry_at<kSym>(slab, a.slab_k, a, jb, rp_nxt, sk, jb.e0 + kWave + lane) : jb.i0 + rp_nxt.r;
        auto batch = [&](const Stage& cur, Stage& nxt, int32_t eb) {
            // requests for the next batches: past the chunk's last entry a
            // lane pairs its row's particle with itself (the entry i decodes
            // to j = i, code 0), so no branch guards them and no register
            // copy at a join has to wait for a load in flight
            nxt.rp = rp_nxt;
            nxt.i = jb.i0 + nxt.rp.r;
            nxt.j = entry_j(raw_nxt, coded);
            nxt.code = entry_code(raw_nxt, coded);
            nxt.in = load_pair(a, src, nxt.i, nxt.j, coded);
            const int32_t e2 = eb + 2 * kWave + lane;
            rp_nxt = row_pos(jb, eb + 2 * kWave, lane, s_mark);
            raw_nxt = e2 < jb.e1 ? entry_at<kSym>(slab, a.slab_k, a, jb, rp_nxt, sk, e2) : jb.i0 + rp_nxt.r;
            const bool valid = eb + lane < jb.e1;
            float px, py, pz, pp;
            bool hit;
            if constexpr (kB) {
                hit = pair32<kWMode, true>(pp_sys, wt, wt + kTab, wt + 2 * kTab, offs, skin, a, cur.in, N, cur.i,
                                           cur.j, cur.code, coded, valid, step, px, py, pz, pp);
            } else {
                hit = pair32<kWMode, true>(kp, s_a, s_g, s_s, offs, skin, a, cur.in, N, cur.i, cur.j, cur.code,
                                           coded, valid, step, px, py, pz, pp);
            }
            float pn = hit ? 1.f : 0.f;
            np_tot += hit ? 1 : 0;
            pe_tot += pp;
            if constexpr (kSym) {
                // a pair inside the chunk: the upper particle's share
                if (hit && (uint32_t)(cur.j - jb.i0) < (uint32_t)jb.ni_once) {
                    const int q = wbase + (cur.j - jb.i0);
                    atomicAdd(&s_jx[q], -px);
                    atomicAdd(&s_jy[q], -py);
                    atomicAdd(&s_jz[q], -pz);
                    if (want_pe) atomicAdd(&s_jp[q], pp);
                    if (want_np) atomicAdd(&s_jn[q], 1);
                    np_tot += 1;
                    pe_tot += pp;
                }
            }
            // the FP32 prefix values stay within a few hundred, so a row's
            // part, their difference, carries an error of a few ulp of that
            px = wave_prefix(px);
            py = wave_prefix(py);
            pz = wave_prefix(pz);
            if (want_pe) pp = wave_prefix(pp);
            if (want_np) pn = wave_prefix(pn);
            const int32_t src = row_end_lane(jb, eb);
            const int32_t first = jb.rstart - eb;
            const float tx = row_part(px, first, src), ty = row_part(py, first, src), tz = row_part(pz, first, src);
            const float tp2 = want_pe ? row_part(pp, first, src) : 0.f;
            const float tn = want_np ? row_part(pn, first, src) : 0.f;
            if (src >= 0) {
                two_sum_add(sx, cx, tx);
                two_sum_add(sy, cy, ty);
                two_sum_add(sz, cz, tz);
                pe_row += tp2;
                np_row += tn;
            }
        };
        for (int32_t eb = jb.e0; eb < jb.e1; eb += 2 * kWave) {
            batch(A, B, eb);
            if (eb + kWave >= jb.e1) break;
            batch(B, A, eb + kWave);
        }
        float jx = 0.f, jy = 0.f, jz = 0.f, jp = 0.f;
        int32_t jn = 0;
        if constexpr (kSym) {
            // LDS operations of one wave take effect in program order: the
            // reads see every atomic above; the slots are cleared for the
            // next chunk
            __asm__ __volatile__("" ::: "memory");
            jx = s_jx[threadIdx.x]; jy = s_jy[threadIdx.x]; jz = s_jz[threadIdx.x];
            jp = s_jp[threadIdx.x]; jn = s_jn[threadIdx.x];
            s_jx[threadIdx.x] = 0.f; s_jy[threadIdx.x] = 0.f; s_jz[threadIdx.x] = 0.f;
            s_jp[threadIdx.x] = 0.f; s_jn[threadIdx.x] = 0;
            __asm__ __volatile__("" ::: "memory");
        }
        if (lane < jb.ni) {
            const int32_t i = jb.i0 + lane;
            double fx = (double)sx + (double)cx, fy = (double)sy + (double)cy, fz = (double)sz + (double)cz;
            if constexpr (kSym) { fx += (double)jx; fy += (double)jy; fz += (double)jz; }
            double pe_b = 0.0;
            if constexpr (kB) {
                const KParams& P = bv.kps[jb.sys];
                if (P.partner || P.body_g != 0.0)
                    add_bonds_body(P, a, i, a.x[i], a.x[N + i], a.x[2 * N + i], fx, fy, fz, pe_b);
            } else {
                if (kp.partner || kp.body_g != 0.0)
                    add_bonds_body(kp, a, i, a.x[i], a.x[N + i], a.x[2 * N + i], fx, fy, fz, pe_b);
            }
            pe_tot += pe_b;
            a.f[i] = fx;
            a.f[N + i] = fy;
            a.f[2 * N + i] = fz;
            if (want_pe) a.pe[i] = (double)pe_row + (double)jp + pe_b;
            if (want_np) a.npair[i] = (int32_t)np_row + jn;
            if constexpr (kVV) vv_row(kp, a, N, i, vin, fx, fy, fz, s_vacc + threadIdx.x);
        }
    }
    if (a.fred_part) block_partials2(pe_tot, 0.5 * (double)np_tot, a.fred_part);
    if constexpr (kVV) vv_partials(s_vacc, a.vv_part);
}

}  // namespace

namespace {
std::atomic<int> g_pair_mode{2};
}  // namespace

// 0: every entry, 1: pairs once, 2: pairs once in the FP64 form only (its
// pair arithmetic outweighs the shorter walk; the mixed walk over the kept
// entries is measured slower than the full one)
bool pairs_once_default(int precision)
{
    const int m = g_pair_mode.load(std::memory_order_relaxed);
    return m == 2 ? precision == 0 : m == 1;
}
int set_pair_mode(int mode) { return g_pair_mode.exchange(mode); }
int pair_mode() { return g_pair_mode.load(std::memory_order_relaxed); }

// Persistent grid: twice the workgroups the chip holds at once (occupancy of
// the kernel times the compute units, cached per device and precision),
// never more than there are 64-particle chunks to hand out.  The second
// round of workgroups starts as the first finishes and keeps every SIMD fed
// through the uneven tails (measured faster than one resident round).
int force_blocks(int32_t n, int precision)
{
    static int cache[16][2] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) dev = 0;
    const int pr = precision ? 1 : 0;
    if (cache[dev][pr] == 0) {
        int per_cu = 0, cus = 0;
        const void* f = pr ? reinterpret_cast<const void*>(&k_force_mixed<0, false, false, false>)
                           : reinterpret_cast<const void*>(&k_force_fp64<0, false, true, false>);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kBlock, 0) != hipSuccess || per_cu < 1)
            per_cu = 4;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        const int full = 2 * per_cu * cus;
        cache[dev][pr] = full < kMaxForceGrid ? full : kMaxForceGrid;
    }
    const int chunks = ceil_div(n > 0 ? n : 1, kChunk);
    const int blocks = ceil_div(chunks, kBlock / kWave);
    return blocks < cache[dev][pr] ? blocks : cache[dev][pr];
}

namespace {

template <bool kB, bool kSym>
void launch_mixed_t(const KParams& kp, const BatchView& bv, const ForceArgs& a, int32_t chunks, dim3 grid,
                    hipStream_t s)
{
    const dim3 block(kBlock);
    switch (kp.wmode) {
    case 0: hipLaunchKernelGGL((k_force_mixed<0, kB, kSym, false>), grid, block, 0, s, kp, bv, a, chunks); break;
    case 1: hipLaunchKernelGGL((k_force_mixed<1, kB, kSym, false>), grid, block, 0, s, kp, bv, a, chunks); break;
    case 2: hipLaunchKernelGGL((k_force_mixed<2, kB, kSym, false>), grid, block, 0, s, kp, bv, a, chunks); break;
    default: hipLaunchKernelGGL((k_force_mixed<3, kB, kSym, false>), grid, block, 0, s, kp, bv, a, chunks); break;
    }
}

template <bool kB, bool kSym>
void launch_forces_t(const KParams& kp, const BatchView& bv, int precision, const ForceArgs& a, hipStream_t s)
{
    const dim3 grid(force_grid(a)), block(kBlock);
    const int32_t chunks = bv.kps ? bv.n_chunks : ceil_div(a.n, kChunk);
    if (precision == 0) {
        if constexpr (!kB) {
            if (a.vv_part) {
                switch (kp.wmode) {
                case 0: hipLaunchKernelGGL((k_force_fp64<0, false, kSym, true>), grid, block, 0, s, kp, bv, a, chunks); break;
                case 1: hipLaunchKernelGGL((k_force_fp64<1, false, kSym, true>), grid, block, 0, s, kp, bv, a, chunks); break;
                case 2: hipLaunchKernelGGL((k_force_fp64<2, false, kSym, true>), grid, block, 0, s, kp, bv, a, chunks); break;
                default: hipLaunchKernelGGL((k_force_fp64<3, false, kSym, true>), grid, block, 0, s, kp, bv, a, chunks); break;
                }
                return;
            }
        }
        switch (kp.wmode) {
        case 0: hipLaunchKernelGGL((k_force_fp64<0, kB, kSym>), grid, block, 0, s, kp, bv, a, chunks); break;
        case 1: hipLaunchKernelGGL((k_force_fp64<1, kB, kSym>), grid, block, 0, s, kp, bv, a, chunks); break;
        case 2: hipLaunchKernelGGL((k_force_fp64<2, kB, kSym>), grid, block, 0, s, kp, bv, a, chunks); break;
        default: hipLaunchKernelGGL((k_force_fp64<3, kB, kSym>), grid, block, 0, s, kp, bv, a, chunks); break;
        }
    } else if constexpr (!kB) {
        if (a.vv_part) {
            switch (kp.wmode) {
            case 0: hipLaunchKernelGGL((k_force_mixed<0, false, kSym, true>), grid, block, 0, s, kp, bv, a, chunks); break;
            case 1: hipLaunchKernelGGL((k_force_mixed<1, false, kSym, true>), grid, block, 0, s, kp, bv, a, chunks); break;
            case 2: hipLaunchKernelGGL((k_force_mixed<2, false, kSym, true>), grid, block, 0, s, kp, bv, a, chunks); break;
            default: hipLaunchKernelGGL((k_force_mixed<3, false, kSym, true>), grid, block, 0, s, kp, bv, a, chunks); break;
            }
            return;
        }
        launch_mixed_t<false, kSym>(kp, bv, a, chunks, grid, s);
    } else {
        launch_mixed_t<true, kSym>(kp, bv, a, chunks, grid, s);
    }
}

}  // namespace

hipError_t launch_skin_filter(const KParams& kp, int precision, const ForceArgs& a, int32_t* kept, int32_t* count,
                              int32_t* kept_flag, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    // a wave per 64-row chunk over a grid of at most 8,192 workgroups
    const int blocks = ceil_div(ceil_div(a.n, kChunk), kBlock / kWave);
    const dim3 grid(blocks < 8192 ? blocks : 8192), block(kBlock);
    // (whether the slab's entries carry stencil codes is known here; with
    // the slab unusable at run time the kernel passes the rows unfiltered)
    const bool coded = a.slab_coded != 0;
    if (precision == 0) {
        if (coded) hipLaunchKernelGGL((k_skin_filter<false, true>), grid, block, 0, s, kp, a, kept, count, kept_flag);
        else hipLaunchKernelGGL((k_skin_filter<false, false>), grid, block, 0, s, kp, a, kept, count, kept_flag);
    } else {
        if (coded) hipLaunchKernelGGL((k_skin_filter<true, true>), grid, block, 0, s, kp, a, kept, count, kept_flag);
        else hipLaunchKernelGGL((k_skin_filter<true, false>), grid, block, 0, s, kp, a, kept, count, kept_flag);
    }
    return hipGetLastError();
}

// In a batch the weight exponent (and so kp.wmode) is shared by all systems.
hipError_t launch_forces(const KParams& kp, const BatchView& bv, int precision, const ForceArgs& a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const bool once = a.pairs_once < 0 ? pairs_once_default(precision) : a.pairs_once != 0;
    if (bv.kps) {
        if (once) launch_forces_t<true, true>(kp, bv, precision, a, s);
        else launch_forces_t<true, false>(kp, bv, precision, a, s);
    } else {
        if (once) launch_forces_t<false, true>(kp, bv, precision, a, s);
        else launch_forces_t<false, false>(kp, bv, precision, a, s);
    }
    return hipGetLastError();
}

}  // namespace dpd
