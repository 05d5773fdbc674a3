// dpd_api.hip -- the C ABI of libdpd (declared in include/dpd.h).
//
// Host-side work only: argument validation, derived parameters, workspace
// carving and the order in which the kernels of one time step are enqueued.
// No entry point synchronises, allocates device memory or throws.
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <utility>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dpd.h"
#include "dpd_launch.h"

namespace dpd {

namespace {

thread_local std::string g_error;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* where)
{
    return fail(DPD_EHIP, "%s: %s", where, hipGetErrorString(e));
}

#define DPD_TRY(expr, where)                          \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

bool finite(double v) { return std::isfinite(v); }

// Cells per side: floor(L / r_list), reduced while a cell would be narrower
// than r_list (1 + 2^-40) so no pair within r_list can sit two cells apart
// once positions and products are rounded.
int cells_per_side(double L, double r_list, int32_t* out)
{
    if (!(L > 0.0) || !(r_list > 0.0) || !finite(L) || !finite(r_list)) return DPD_EINVAL;
    const double q = std::floor(L / r_list);
    if (q > 4096.0) return DPD_EINVAL;
    int32_t m = (int32_t)q;
    const double min_side = r_list * (1.0 + std::ldexp(1.0, -40));
    while (m > 0 && L / (double)m < min_side) --m;
    if (m < 3 || m > 1023) return DPD_EINVAL;
    *out = m;
    return DPD_OK;
}

int make_kparams(const dpd_params* p, KParams* k)
{
    if (!p) return fail(DPD_EINVAL, "params is NULL");
    std::memset(k, 0, sizeof(*k));
    if (!(p->r_c > 0.0) || !finite(p->r_c)) return fail(DPD_EINVAL, "r_c must be > 0");
    if (!(p->skin >= 0.0) || !finite(p->skin)) return fail(DPD_EINVAL, "skin must be >= 0");
    if (!(p->dt > 0.0) || !finite(p->dt)) return fail(DPD_EINVAL, "dt must be > 0");
    if (!(p->s > 0.0) || !finite(p->s)) return fail(DPD_EINVAL, "s must be > 0");
    if (!finite(p->lambda)) return fail(DPD_EINVAL, "lambda must be finite");
    if (p->n_types < 1 || p->n_types > DPD_MAX_TYPES) return fail(DPD_EINVAL, "n_types must be in [1, %d]", DPD_MAX_TYPES);
    const double r_list = p->r_c + p->skin;
    for (int d = 0; d < 3; ++d) {
        if (cells_per_side(p->box[d], r_list, &k->nc[d]) != DPD_OK)
            return fail(DPD_EINVAL, "box[%d] = %g gives fewer than 3 (or more than 1023) cells of side >= %g",
                        d, p->box[d], r_list);
        k->L[d] = p->box[d];
        k->halfL[d] = 0.5 * p->box[d];
        k->inv_cell[d] = (double)k->nc[d] / p->box[d];
        k->cell_len[d] = p->box[d] / (double)k->nc[d];
        k->cell_len32[d] = (float)k->cell_len[d];
        k->L32[d] = (float)p->box[d];
    }
    const int64_t ncell = (int64_t)k->nc[0] * k->nc[1] * k->nc[2];
    if (ncell >= (int64_t)1 << 31) return fail(DPD_EINVAL, "too many cells");
    k->n_cells = (int32_t)ncell;
    int32_t nmax = k->nc[0] > k->nc[1] ? k->nc[0] : k->nc[1];
    nmax = nmax > k->nc[2] ? nmax : k->nc[2];
    k->nbits = bits_for(nmax);
    int32_t bmax = 1;
    int64_t nblk = 1;
    for (int d = 0; d < 3; ++d) {
        k->nb[d] = (k->nc[d] + 1) / 2;
        k->small_dim[d] = k->nc[d] < 4 ? 1 : 0;
        bmax = k->nb[d] > bmax ? k->nb[d] : bmax;
        nblk *= k->nb[d];
    }
    k->nbits_b = bits_for(bmax);
    k->n_blocks = (int32_t)nblk;
    const int32_t tdim[3] = {kTileX, kTileY, kTileZ};
    int64_t ntile = 1;
    for (int d = 0; d < 3; ++d) {
        k->nt[d] = (k->nc[d] + tdim[d] - 1) / tdim[d];
        ntile *= k->nt[d];
    }
    k->n_tiles = (int32_t)ntile;
    k->rl2 = r_list * r_list;
    // FP32 separations from cell offsets are within ~3e-6 r_list^2 of the
    // FP64 value (offsets below 4 cells); the band is ten times wider
    k->list_lo32 = (float)(k->rl2 * (1.0 - std::ldexp(1.0, -15)));
    k->list_hi32 = (float)(k->rl2 * (1.0 + std::ldexp(1.0, -15)));
    // tile-frame positions reach 6 cell lengths from the frame origin: FP32
    // separations are within ~2e-5 r_list^2 there; the band is ~6x wider
    k->tile_lo32 = (float)(k->rl2 * (1.0 - std::ldexp(1.0, -13)));
    k->tile_hi32 = (float)(k->rl2 * (1.0 + std::ldexp(1.0, -13)));
    k->rc2 = p->r_c * p->r_c;
    k->r_c = p->r_c;
    k->inv_rc = 1.0 / p->r_c;
    k->dt = p->dt;
    k->half_dt = 0.5 * p->dt;
    k->lam_dt = p->lambda * p->dt;
    k->lam_half = (p->lambda == 0.5) ? 1 : 0;
    k->s = p->s;
    k->wmode = (p->s == 0.5) ? 0 : (p->s == 1.0) ? 1 : (p->s == 2.0) ? 2 : 3;
    const int nt = p->n_types;
    k->n_types = nt;
    const double rdt = 1.0 / std::sqrt(p->dt);
    for (int t = 0; t < nt; ++t)
        for (int u = 0; u < nt; ++u) {
            const int tu = t * nt + u, ut = u * nt + t;
            const double a = p->a[tu], g = p->gamma[tu], sg = p->sigma[tu];
            if (!finite(a) || !finite(g) || !finite(sg))
                return fail(DPD_EINVAL, "non-finite a / gamma / sigma at (%d, %d)", t, u);
            if (a != p->a[ut] || g != p->gamma[ut] || sg != p->sigma[ut])
                return fail(DPD_EINVAL, "a / gamma / sigma must be symmetric (entry (%d, %d))", t, u);
            k->a[tu] = a;
            k->g[tu] = g;
            k->srdt[tu] = sg * rdt;
        }
    k->seed_lo = (uint32_t)p->seed;
    k->seed_hi = (uint32_t)(p->seed >> 32);
    if (!finite(p->body_g) || !finite(p->body_split)) return fail(DPD_EINVAL, "body force must be finite");
    k->body_g = p->body_g;
    k->body_split = p->body_split;
    if (p->bond_partner && (!finite(p->bond_k) || !finite(p->bond_r0)))
        return fail(DPD_EINVAL, "bond parameters must be finite");
    k->bond_k = p->bond_k;
    k->bond_r0 = p->bond_r0;
    k->partner = p->bond_partner;
    return DPD_OK;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

bool aligned(const void* ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

int check_state(const dpd_state* s, const char* name, bool need_f)
{
    if (!s) return fail(DPD_EINVAL, "%s is NULL", name);
    if (s->n < 0) return fail(DPD_EINVAL, "%s->n must be >= 0", name);
    if (s->n == 0) return DPD_OK;
    if (!s->x || !s->v || !s->tag || !s->type || (need_f && !s->f))
        return fail(DPD_EINVAL, "%s has a NULL array", name);
    if (!aligned(s->x, 8) || !aligned(s->v, 8) || (s->f && !aligned(s->f, 8)) || !aligned(s->tag, 4))
        return fail(DPD_EINVAL, "%s arrays are misaligned", name);
    return DPD_OK;
}

int check_ws(void* ws, size_t ws_bytes, size_t need)
{
    if (need == 0) return DPD_OK;
    if (!ws) return fail(DPD_EINVAL, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(DPD_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(DPD_ECAPACITY, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    return DPD_OK;
}

template <typename T>
T* carve(void* ws, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(ws) + off); }

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

// What one enqueue covers: a single system (bv.kps == nullptr) or a batch.
struct Job {
    KParams kp;          // the system (single) or the shared fields of a batch
    BatchView bv;
    int32_t n_cells;     // cells of all systems
    int32_t n_blocks;    // 2x2x2 list blocks of all systems
    int32_t n_tiles;     // list-build tiles of all systems
    int32_t slab_k;      // neighbour slab width
    int32_t force_grid;  // persistent force workgroups (0 = default)
    int32_t nlist_waves; // waves per list-build workgroup
    int32_t nlist_kind;  // 0: tile builder, 1: wave per 2x2x2 cell block, 2: lane per particle
    Gate gate = nullptr; // skin steps: rebuild only while *gate != 0
};

// the list builder of single-system calls (dpd_set_list_builder)
std::atomic<int> g_list_builder{0};

Job single_job(const KParams& kp, int32_t n)
{
    Job j;
    j.kp = kp;
    std::memset(&j.bv, 0, sizeof(j.bv));
    j.n_cells = kp.n_cells;
    j.n_blocks = kp.n_blocks;
    j.n_tiles = kp.n_tiles;
    const double vol = kp.L[0] * kp.L[1] * kp.L[2];
    j.slab_k = nlist_slab_width(n / vol, kp.rl2);
    j.force_grid = 0;
    j.nlist_waves = 4;
    j.nlist_kind = g_list_builder.load(std::memory_order_relaxed);
    return j;
}

// aos: also lay out the packed FP64 copies the FP64 step reads (placed
// last, so every other offset is the same either way)
WsLayout ws_layout(const Job& job, int32_t n, bool aos = false)
{
    WsLayout w;
    size_t o = 0;
    const size_t N = (size_t)(n > 0 ? n : 1);
    const bool need_vt = !job.kp.lam_half;
    const int32_t n_cells = job.n_cells;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    w.bx = take(3 * N * sizeof(double));
    w.bv = take(3 * N * sizeof(double));
    w.bvt = need_vt ? take(3 * N * sizeof(double)) : 0;
    w.vt_sorted = need_vt ? take(3 * N * sizeof(double)) : 0;
    w.btag = take(N * sizeof(uint32_t));
    w.btype = take(N);
    w.key = take(N * sizeof(int32_t));
    w.slot = take(N * sizeof(int32_t));
    w.cxyz = take(N * sizeof(uint32_t));
    w.tmp_tag = take(N * sizeof(uint32_t));
    w.tmp_src = take(N * sizeof(int32_t));
    w.tmp_key = take(N * sizeof(int32_t));
    const int64_t scan_items = (int64_t)(n > n_cells ? n : n_cells) + 1;
    w.scan_part = take((size_t)ceil_div(scan_items, kScanTile) * sizeof(int32_t) + 64);
    w.rank_tab = take((size_t)(n_cells > 0 ? n_cells : 1) * sizeof(int32_t));
    w.slab_k = job.slab_k;
    w.slab = take(N * (size_t)w.slab_k * sizeof(int32_t));
    w.slab_flag = take(sizeof(int32_t));
    // (momentum and |v|^2 partials: kRedBlocks of them from the integration
    // kernels, one per force workgroup from the force pass's epilogue)
    w.red_part = take((size_t)3 * (kRedBlocks > kMaxForceGrid ? kRedBlocks : kMaxForceGrid) * 2 * sizeof(double));
    w.fred_part = take((size_t)kMaxForceGrid * 2 * sizeof(double));
    w.fsum_part = take((size_t)kRedBlocks * 2 * sizeof(double));
    w.bwd_part = take((size_t)backward_part_doubles(n, job.kp.n_types) * sizeof(double));
    // per-particle potential energy and pair counts (per-system statistics of a batch)
    w.pe_part = take(N * sizeof(double));
    w.np_part = take(N * sizeof(int32_t));
    w.sys_part = take((size_t)(job.bv.kps && job.bv.n_chunks > 0 ? job.bv.n_chunks : 1) * 6 * sizeof(double));
    w.tile_rest = take(((size_t)(job.n_tiles > 0 ? job.n_tiles : 0) + 1) * sizeof(int32_t));
    const bool bonds = job.kp.partner != nullptr;
    w.pidx_a = bonds ? take(2 * N * sizeof(int32_t)) : 0;
    w.pidx_b = bonds ? take(2 * N * sizeof(int32_t)) : 0;
    w.inv = bonds ? take(N * sizeof(int32_t)) : 0;
    const bool skin = job.kp.rl2 != job.kp.rc2;
    w.xref = skin ? take(3 * N * sizeof(double)) : 0;
    w.gate = skin ? take(2 * sizeof(int32_t)) : 0;
    w.kept = skin ? take(N * (size_t)w.slab_k * sizeof(int32_t)) : 0;
    w.kept_off = skin ? take((N + 1) * sizeof(int32_t)) : 0;
    w.kept_flag = skin ? take(sizeof(int32_t)) : 0;
    w.x64 = aos ? take(N * 4 * sizeof(double)) : 0;
    w.v64 = aos ? take(N * 4 * sizeof(double)) : 0;
    w.total = o;
    return w;
}

WsLayout ws_layout(const KParams& kp, int32_t n, bool aos) { return ws_layout(single_job(kp, n), n, aos); }

namespace {

// binning + reordering from `in` into `out` (shared by dpd_bin_reorder and dpd_step)
int enqueue_reorder(const Job& job, const WsLayout& L, void* ws, const dpd_state* in,
                    const double* vt_in, dpd_state* out, double* vt_out, dpd_cells* cells,
                    float* x32, float* v32, hipStream_t s, bool aos = false, int32_t* inv = nullptr,
                    bool write_iot = true)
{
    const int32_t n = in->n;
    int32_t* key = carve<int32_t>(ws, L.key);
    int32_t* slot = carve<int32_t>(ws, L.slot);
    uint32_t* cxyz = carve<uint32_t>(ws, L.cxyz);
    uint32_t* tmp_tag = carve<uint32_t>(ws, L.tmp_tag);
    int32_t* tmp_src = carve<int32_t>(ws, L.tmp_src);
    int32_t* tmp_key = carve<int32_t>(ws, L.tmp_key);
    int32_t* part = carve<int32_t>(ws, L.scan_part);
    const int32_t* rank_tab = carve<int32_t>(ws, L.rank_tab);
    const Gate gt = job.gate;
    DPD_TRY(launch_fill_i32(cells->cell_start, (int64_t)job.n_cells + 1, 0, s, gt), "fill cell counts");
    DPD_TRY(launch_bin(job.kp, job.bv, n, in->x, rank_tab, key, slot, cxyz, cells->cell_start, s, gt), "bin");
    DPD_TRY(launch_scan(cells->cell_start, (int64_t)job.n_cells + 1, part, s, gt), "scan cells");
    DPD_TRY(launch_place(n, key, slot, cells->cell_start, in->tag, tmp_tag, tmp_src, tmp_key, s, gt), "place");
    GatherArgs g;
    g.x_in = in->x; g.v_in = in->v; g.vt_in = vt_in; g.type_in = in->type; g.cxyz_in = cxyz;
    g.x_out = out->x; g.v_out = out->v; g.vt_out = vt_out; g.tag_out = out->tag; g.type_out = out->type;
    g.cell_xyz = cells->cell_xyz; g.perm = cells->perm; g.idx_of_tag = write_iot ? cells->idx_of_tag : nullptr;
    g.inv = inv;
    g.x32 = x32; g.v32 = v32;
    g.x64 = aos ? carve<double>(ws, L.x64) : nullptr;
    g.v64 = aos ? carve<double>(ws, L.v64) : nullptr;
    g.xref = job.gate ? carve<double>(ws, L.xref) : nullptr;
    DPD_TRY(launch_finalize(job.kp, job.bv, n, tmp_key, cells->cell_start, tmp_tag, tmp_src, g, s, gt), "finalize");
    return DPD_OK;
}

int enqueue_nlist(const Job& job, const WsLayout& L, void* ws, const dpd_state* st,
                  const dpd_cells* cells, const float* x32, dpd_nlist* nl, int32_t* d_status, hipStream_t s,
                  bool compact = true)
{
    DPD_TRY(launch_nlist(job.kp, job.bv, job.n_cells, job.n_blocks, job.n_tiles, st->n, st->x, x32, cells->cell_xyz,
                         cells->cell_start, carve<int32_t>(ws, L.rank_tab), nl->offset, nl->index, nl->capacity,
                         carve<int32_t>(ws, L.slab), L.slab_k, carve<int32_t>(ws, L.slab_flag),
                         carve<int32_t>(ws, L.tile_rest), d_status,
                         carve<int32_t>(ws, L.scan_part), job.nlist_waves, job.nlist_kind, compact, s, job.gate),
            "neighbour list");
    return DPD_OK;
}

int enqueue_rank_table(const Job& job, const WsLayout& L, void* ws, hipStream_t s)
{
    DPD_TRY(launch_rank_table(job.kp, job.bv, job.n_cells, carve<int32_t>(ws, L.rank_tab), s), "rank table");
    return DPD_OK;
}

int check_cells(const dpd_cells* c, int32_t n, bool need_iot)
{
    if (!c) return fail(DPD_EINVAL, "cells is NULL");
    if (!c->cell_start) return fail(DPD_EINVAL, "cells->cell_start is NULL");
    if (n > 0 && (!c->cell_xyz || !c->perm)) return fail(DPD_EINVAL, "cells arrays are NULL");
    if (n > 0 && need_iot && !c->idx_of_tag) return fail(DPD_EINVAL, "bonds need cells->idx_of_tag");
    return DPD_OK;
}

int check_nlist(const dpd_nlist* nl, int32_t n)
{
    if (!nl) return fail(DPD_EINVAL, "nlist is NULL");
    if (!nl->offset) return fail(DPD_EINVAL, "nlist->offset is NULL");
    if (nl->capacity < 0 || nl->capacity >= ((int64_t)1 << 31))
        return fail(DPD_EINVAL, "nlist capacity must be in [0, 2^31)");
    if (n > 0 && nl->capacity > 0 && !nl->index) return fail(DPD_EINVAL, "nlist->index is NULL");
    return DPD_OK;
}

// ---------------------------------------------------------------------------
// Batched replicas
// ---------------------------------------------------------------------------

// Device table of a batch (caller memory): per-system KParams, the particle /
// cell / block offsets, the particle -> system map and a step-counter
// snapshot that numbers the rows of the per-step statistics.
struct BatchTable {
    size_t kps, p_off, c_off, b_off, t_off, ch_off, sys_of, step_base, total;
};

BatchTable batch_table(int32_t n_sys, int64_t n_total)
{
    BatchTable t;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    const size_t ns = (size_t)n_sys;
    t.kps = take(ns * sizeof(KParams));
    t.p_off = take((ns + 1) * sizeof(int32_t));
    t.c_off = take((ns + 1) * sizeof(int32_t));
    t.b_off = take((ns + 1) * sizeof(int32_t));
    t.t_off = take((ns + 1) * sizeof(int32_t));
    t.ch_off = take((ns + 1) * sizeof(int32_t));
    t.sys_of = take((size_t)(n_total > 0 ? n_total : 1) * sizeof(uint16_t));
    t.step_base = take(sizeof(uint64_t));
    t.total = o;
    return t;
}

// Arguments a captured step depends on; a change means capturing again.
struct GraphKey {
    int32_t precision;
    int32_t force_grid, nlist_waves, nlist_kind, pairs_once;
    dpd_state st;
    dpd_cells cells;
    dpd_nlist nl;
    const void *d_step, *red, *x32, *v32, *d_status, *ws;
    size_t ws_bytes;
};

}  // namespace
}  // namespace dpd

struct dpd_batch {
    int32_t n_sys = 0;
    int64_t n_total = 0;
    dpd::Job job;                      // shared KParams (system 0) + BatchView + totals + tiles
    std::vector<dpd::KParams> kps;     // host copies (the device table is filled from these)
    std::vector<int32_t> p_off, c_off, b_off, t_off, ch_off;
    uint64_t* step_base = nullptr;     // device
    hipGraphExec_t exec = nullptr;     // cached one-step graph
    hipStream_t capture = nullptr;     // stream the graph is captured on
    dpd::GraphKey key;
    bool have_key = false;
};

namespace dpd {
namespace {

void drop_graph(dpd_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->have_key = false;
}

int check_batch_state(const dpd_batch* b, const dpd_state* st, const char* name, bool need_f)
{
    const int rc = check_state(st, name, need_f);
    if (rc) return rc;
    if ((int64_t)st->n != b->n_total)
        return fail(DPD_EINVAL, "%s->n = %d but the batch holds %lld particles", name, st->n,
                    (long long)b->n_total);
    return DPD_OK;
}

// one batched step: integrate, reorder, list, forces, integrate, statistics
// One batched step.  The force pass reads the builder's slab rows; the CSR
// index is written by dpd_batch_step once, after its last step.
int enqueue_batch_step(const dpd_batch* bt, const WsLayout& L, void* ws, int32_t precision, dpd_state* st,
                       uint64_t* d_step, double* red, dpd_cells* cells, dpd_nlist* nl, float* x32, float* v32,
                       int32_t* d_status, hipStream_t s)
{
    const Job& job = bt->job;
    const KParams& kp = job.kp;
    const int32_t n = st->n;
    dpd_state b;                                    // drifted, not yet reordered
    b.n = n;
    b.x = carve<double>(ws, L.bx);
    b.v = carve<double>(ws, L.bv);
    b.f = nullptr;
    b.tag = carve<uint32_t>(ws, L.btag);
    b.type = carve<uint8_t>(ws, L.btype);
    double* bvt = kp.lam_half ? nullptr : carve<double>(ws, L.bvt);
    double* vt_sorted = kp.lam_half ? nullptr : carve<double>(ws, L.vt_sorted);
    const bool mixed = precision == DPD_MIXED;
    ForceArgs a;
    a.n = n; a.x = st->x; a.v = kp.lam_half ? st->v : vt_sorted; a.tag = st->tag; a.type = st->type;
    a.cell_xyz = cells->cell_xyz; a.x32 = x32; a.v32 = v32;
    a.offset = nl->offset; a.index = nl->index; a.capacity = nl->capacity;
    a.idx_of_tag = cells->idx_of_tag;
    a.d_step = d_step; a.step_add = 1;
    a.f = st->f;
    a.pe = carve<double>(ws, L.pe_part);
    a.npair = carve<int32_t>(ws, L.np_part);
    a.fred_part = nullptr;
    a.status = d_status;
    a.grid = job.force_grid > 0 ? job.force_grid : force_blocks(n, precision);
    a.slab = carve<int32_t>(ws, L.slab);
    a.slab_k = L.slab_k;
    a.slab_flag = carve<int32_t>(ws, L.slab_flag);
    a.slab_coded = nlist_slab_coded(job.nlist_kind, cells->cell_xyz, job.n_cells, n) ? 1 : 0;
    const bool aos = precision == DPD_FP64;
    a.x64 = aos ? carve<double>(ws, L.x64) : nullptr;
    a.v64 = aos ? carve<double>(ws, L.v64) : nullptr;
    int rc;
    DPD_TRY(launch_vv1(kp, job.bv, n, st->x, st->v, st->f, st->tag, st->type, b.x, b.v, bvt, b.tag, b.type, s),
            "vv1");
    if ((rc = enqueue_reorder(job, L, ws, &b, bvt, st, vt_sorted, cells, x32, mixed ? v32 : nullptr, s, aos)))
        return rc;
    if ((rc = enqueue_nlist(job, L, ws, st, cells, x32, nl, d_status, s, false))) return rc;
    DPD_TRY(launch_forces(kp, job.bv, precision, a, s), "forces");
    // the second half-kick (dt is shared by the systems) and the statistics
    // in one pass per 64-particle chunk
    DPD_TRY(launch_sys_reduce(job.bv, n, st->v, st->f, kp.half_dt, a.pe, a.npair, carve<double>(ws, L.sys_part),
                              red, d_step, bt->step_base, d_status, s),
            "vv2 + system statistics");
    DPD_TRY(launch_counter(d_step, nullptr, s), "step counter");
    return DPD_OK;
}

// Argument checks and kernel arguments shared by the force entry points
// (everything except where the per-workgroup partials go).
int prepare_forces(const dpd_params* p, int32_t precision, const dpd_state* sorted, const dpd_cells* cells,
                   const float* x32, const float* v32, const dpd_nlist* nl, uint64_t step, double* f_out,
                   double* pe_out, int32_t* d_status, KParams* kp_out, ForceArgs* out)
{
    KParams& kp = *kp_out;
    int rc = make_kparams(p, &kp);
    if (rc) return rc;
    if (precision != DPD_FP64 && precision != DPD_MIXED) return fail(DPD_EINVAL, "unknown precision %d", precision);
    if ((rc = check_state(sorted, "sorted", false))) return rc;
    const int32_t n = sorted->n;
    if ((rc = check_nlist(nl, n))) return rc;
    if (n > 0 && !f_out) return fail(DPD_EINVAL, "f_out is NULL");
    const bool bonds = kp.partner != nullptr;
    if (bonds && (rc = check_cells(cells, n, true))) return rc;
    if (precision == DPD_MIXED && n > 0 && (!x32 || !v32))
        return fail(DPD_EINVAL, "mixed precision needs x32 and v32");
    if (precision == DPD_MIXED && n > 0 && (!aligned(x32, 16) || !aligned(v32, 16)))
        return fail(DPD_EINVAL, "x32 / v32 must be 16-byte aligned");
    ForceArgs& a = *out;
    a.n = n; a.x = sorted->x; a.v = sorted->v; a.tag = sorted->tag; a.type = sorted->type;
    a.cell_xyz = cells ? cells->cell_xyz : nullptr; a.x32 = x32; a.v32 = v32;
    a.offset = nl->offset; a.index = nl->index; a.capacity = nl->capacity;
    a.idx_of_tag = cells ? cells->idx_of_tag : nullptr;
    a.d_step = nullptr; a.step_add = step;
    a.f = f_out; a.pe = pe_out;
    a.npair = nullptr;
    a.fred_part = nullptr;
    a.status = d_status;
    a.grid = force_blocks(n, precision);
    a.slab = nullptr; a.slab_k = 0; a.slab_flag = nullptr; a.slab_coded = 0;
    a.x64 = nullptr; a.v64 = nullptr;
    return DPD_OK;
}

// the force pass and, with stats, the fixed-order sum of its partials
int enqueue_forces(const KParams& kp, int32_t precision, const ForceArgs& a, double* stats, int32_t* d_status,
                   hipStream_t s)
{
    const BatchView none{};
    DPD_TRY(launch_forces(kp, none, precision, a, s), "forces");
    if (stats)
        DPD_TRY(launch_reduce_final(a.n, nullptr, 0, a.fred_part, force_grid(a), nullptr, stats, nullptr,
                                    d_status, s), "force stats");
    return DPD_OK;
}

}  // namespace
}  // namespace dpd

namespace dpd {

// Scratch of dpd_forces_noalloc: the force pass's per-workgroup (potential
// energy, pair count) partials, one pair of doubles per workgroup of the
// largest force grid (kMaxForceGrid), 128 KiB on every device the library
// runs on, held until the process ends.  Host code never passes `scratch`
// itself to a kernel (in host code it names a host-side stand-in): each
// device's address comes from hipGetSymbolAddress, taken once per device
// with that device current.
constexpr size_t kScratchDoubles = (size_t)kMaxForceGrid * 2;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// this device's copy of `scratch` (its address looked up on the first call
// on the device)
int scratch_on_current_device(double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(DPD_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(DPD_EUNSUPPORTED, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(DPD_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return DPD_OK;
}

}  // namespace
}  // namespace dpd

using namespace dpd;

extern "C" {

const char* dpd_last_error(void) { return g_error.c_str(); }

const char* dpd_version(void) { return "libdpd 0.1 (gfx950)"; }

int dpd_set_pair_evaluation(int32_t mode)
{
    if (mode < 0 || mode > 2) return fail(DPD_EINVAL, "pair evaluation mode must be 0, 1 or 2");
    return set_pair_mode(mode);
}

int dpd_set_list_builder(int32_t kind)
{
    if (kind < 0 || kind > 2) return fail(DPD_EINVAL, "list builder kind must be 0, 1 or 2");
    return g_list_builder.exchange(kind);
}

int dpd_cell_grid(const dpd_params* p, int32_t nc[3])
{
    if (!p || !nc) return fail(DPD_EINVAL, "NULL argument");
    KParams k;
    const int rc = make_kparams(p, &k);
    if (rc != DPD_OK) return rc;
    for (int d = 0; d < 3; ++d) nc[d] = k.nc[d];
    return DPD_OK;
}

size_t dpd_workspace_bytes(const dpd_params* p, int32_t n, int32_t precision)
{
    KParams k;
    if (n < 0 || (precision != DPD_FP64 && precision != DPD_MIXED) || make_kparams(p, &k) != DPD_OK) return 0;
    return ws_layout(k, n, precision == DPD_FP64).total;
}

int dpd_bin_reorder(const dpd_params* p, const dpd_state* in, dpd_state* out, dpd_cells* cells,
                    float* x32, float* v32, void* ws, size_t ws_bytes, void* stream)
{
    KParams kp;
    int rc = make_kparams(p, &kp);
    if (rc) return rc;
    if ((rc = check_state(in, "in", false)) || (rc = check_state(out, "out", false))) return rc;
    if (in->n != out->n) return fail(DPD_EINVAL, "in->n != out->n");
    if (in->n > 0 && (in->x == out->x || in->v == out->v || in->tag == out->tag || in->type == out->type))
        return fail(DPD_EINVAL, "in and out must not overlap");
    if ((rc = check_cells(cells, in->n, false))) return rc;
    const Job job = single_job(kp, in->n);
    const WsLayout L = ws_layout(job, in->n);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    if ((rc = enqueue_rank_table(job, L, ws, as_stream(stream)))) return rc;
    return enqueue_reorder(job, L, ws, in, nullptr, out, nullptr, cells, x32, v32, as_stream(stream));
}

int dpd_build_neighbors(const dpd_params* p, const dpd_state* sorted, const dpd_cells* cells,
                        const float* x32, dpd_nlist* nl, int32_t* d_status, void* ws, size_t ws_bytes,
                        void* stream)
{
    KParams kp;
    int rc = make_kparams(p, &kp);
    if (rc) return rc;
    if (!sorted) return fail(DPD_EINVAL, "sorted is NULL");
    if (sorted->n < 0) return fail(DPD_EINVAL, "n must be >= 0");
    if (sorted->n > 0 && !sorted->x) return fail(DPD_EINVAL, "sorted->x is NULL");
    if ((rc = check_cells(cells, sorted->n, false)) || (rc = check_nlist(nl, sorted->n))) return rc;
    if (sorted->n > 0 && !x32) return fail(DPD_EINVAL, "x32 (from dpd_bin_reorder) is NULL");
    const Job job = single_job(kp, sorted->n);
    const WsLayout L = ws_layout(job, sorted->n);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    if ((rc = enqueue_rank_table(job, L, ws, as_stream(stream)))) return rc;
    return enqueue_nlist(job, L, ws, sorted, cells, x32, nl, d_status, as_stream(stream));
}

int dpd_forces(const dpd_params* p, int32_t precision, const dpd_state* sorted, const dpd_cells* cells,
               const float* x32, const float* v32, const dpd_nlist* nl, uint64_t step, double* f_out,
               double* pe_out, double* stats, int32_t* d_status, void* ws, size_t ws_bytes, void* stream)
{
    KParams kp;
    ForceArgs a;
    int rc = prepare_forces(p, precision, sorted, cells, x32, v32, nl, step, f_out, pe_out, d_status, &kp, &a);
    if (rc) return rc;
    const WsLayout L = ws_layout(kp, a.n);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    a.fred_part = stats ? carve<double>(ws, L.fred_part) : nullptr;
    return enqueue_forces(kp, precision, a, stats, d_status, as_stream(stream));
}

int dpd_forces_noalloc(const dpd_params* p, int32_t precision, const dpd_state* sorted, const dpd_cells* cells,
                       const float* x32, const float* v32, const dpd_nlist* nl, uint64_t step, double* f_out,
                       double* pe_out, double* stats, int32_t* d_status, void* stream)
{
    KParams kp;
    ForceArgs a;
    int rc = prepare_forces(p, precision, sorted, cells, x32, v32, nl, step, f_out, pe_out, d_status, &kp, &a);
    if (rc) return rc;
    a.fred_part = nullptr;
    if (stats && a.n > 0) {
        if ((size_t)force_grid(a) * 2 > kScratchDoubles)
            return fail(DPD_ECAPACITY, "force grid of %d workgroups exceeds the scratch of %d", force_grid(a),
                        kMaxForceGrid);
        double* part = nullptr;
        if ((rc = scratch_on_current_device(&part))) return rc;
        a.fred_part = part;                        // every workgroup overwrites its own pair
    }
    return enqueue_forces(kp, precision, a, stats, d_status, as_stream(stream));
}

int dpd_step(const dpd_params* p, int32_t precision, dpd_state* st, int32_t n_steps, uint64_t* d_step,
             double* d_reductions, dpd_cells* cells, dpd_nlist* nl, float* x32, float* v32,
             int32_t* d_status, void* const* phase_events, void* ws, size_t ws_bytes, void* stream)
{
    KParams kp;
    int rc = make_kparams(p, &kp);
    if (rc) return rc;
    if (precision != DPD_FP64 && precision != DPD_MIXED) return fail(DPD_EINVAL, "unknown precision %d", precision);
    if ((rc = check_state(st, "state", true))) return rc;
    if (n_steps < 0) return fail(DPD_EINVAL, "n_steps must be >= 0");
    if (!d_step) return fail(DPD_EINVAL, "d_step is NULL");
    const int32_t n = st->n;
    const bool bonds = kp.partner != nullptr;
    if ((rc = check_cells(cells, n, bonds)) || (rc = check_nlist(nl, n))) return rc;
    if (n > 0 && !x32) return fail(DPD_EINVAL, "x32 is NULL (the list build needs it)");
    if (precision == DPD_MIXED && n > 0 && !v32) return fail(DPD_EINVAL, "mixed precision needs v32");
    const Job job = single_job(kp, n);
    const bool aos = precision == DPD_FP64;
    const WsLayout L = ws_layout(job, n, aos);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    if (n == 0 || n_steps == 0) return DPD_OK;
    const hipStream_t s = as_stream(stream);
    if ((rc = enqueue_rank_table(job, L, ws, s))) return rc;

    dpd_state b;                                    // drifted, not yet reordered
    b.n = n;
    b.x = carve<double>(ws, L.bx);
    b.v = carve<double>(ws, L.bv);
    b.f = nullptr;
    b.tag = carve<uint32_t>(ws, L.btag);
    b.type = carve<uint8_t>(ws, L.btype);
    double* bvt = kp.lam_half ? nullptr : carve<double>(ws, L.bvt);
    double* vt_sorted = kp.lam_half ? nullptr : carve<double>(ws, L.vt_sorted);

    ForceArgs a;
    a.n = n; a.x = st->x; a.v = kp.lam_half ? st->v : vt_sorted; a.tag = st->tag; a.type = st->type;
    a.cell_xyz = cells->cell_xyz; a.x32 = x32; a.v32 = v32;
    a.offset = nl->offset; a.index = nl->index; a.capacity = nl->capacity;
    a.idx_of_tag = cells->idx_of_tag;
    a.d_step = d_step; a.step_add = 1;
    a.f = st->f; a.pe = nullptr; a.npair = nullptr;
    a.fred_part = carve<double>(ws, L.fred_part);
    a.status = d_status;
    a.grid = force_blocks(n, precision);
    a.slab = carve<int32_t>(ws, L.slab);
    a.slab_k = L.slab_k;
    a.slab_flag = carve<int32_t>(ws, L.slab_flag);
    a.slab_coded = nlist_slab_coded(job.nlist_kind, cells->cell_xyz, job.n_cells, n) ? 1 : 0;
    a.x64 = aos ? carve<double>(ws, L.x64) : nullptr;
    a.v64 = aos ? carve<double>(ws, L.v64) : nullptr;
    double* red_part = carve<double>(ws, L.red_part);
    double* fsum_part = carve<double>(ws, L.fsum_part);
    const bool mixed = precision == DPD_MIXED;

    // Bonds: the first reorder of the call writes the tag -> index map and
    // the partners' sorted indices are looked up from it once; later steps
    // carry them from reorder to reorder (coherent gathers instead of a
    // scatter by tag), and the map is written again at the last step.
    int32_t* pidx_cur = bonds ? carve<int32_t>(ws, L.pidx_a) : nullptr;
    int32_t* pidx_nxt = bonds ? carve<int32_t>(ws, L.pidx_b) : nullptr;
    int32_t* inv = bonds ? carve<int32_t>(ws, L.inv) : nullptr;

    auto mark = [&](int32_t k, int phase) -> hipError_t {
        if (!phase_events) return hipSuccess;
        return hipEventRecord(reinterpret_cast<hipEvent_t>(phase_events[6 * (int64_t)k + phase]), s);
    };
    // Phase 2 of step k and phase 1 of step k + 1 run as one pass over the
    // state (v after phase 2 is only needed for the statistics and by the
    // next phase 1); the last step's phase 2 runs alone.
    DriftArgs drift{st->x, st->tag, st->type, b.x, b.v, bvt, b.tag, b.type};
    // With a skin, the first step of the call rebuilds; every later step
    // drifts the sorted state in place and rebuilds (copy to the reorder's
    // source, reorder, list) only when some particle has moved more than
    // skin / 2 since the last rebuild, which the drift pass reports in the
    // step's gate (steps alternate between two gate words, so the statistics
    // of step k - 1, summed during step k, still see their step's word).
    const bool skin = kp.rl2 != kp.rc2;
    int32_t* gates = skin ? carve<int32_t>(ws, L.gate) : nullptr;
    const double half_skin = 0.5 * (p->skin);
    SkinDriftArgs sd;
    sd.x = st->x; sd.v = st->v; sd.vt = vt_sorted; sd.f = st->f;
    sd.tag = st->tag; sd.type = st->type; sd.cell_xyz = cells->cell_xyz;
    sd.xref = skin ? carve<double>(ws, L.xref) : nullptr;
    sd.x32 = mixed ? x32 : nullptr;           // (the FP64 step reads x32 only in a rebuild)
    sd.v32 = mixed ? v32 : nullptr;
    sd.x64 = aos ? carve<double>(ws, L.x64) : nullptr;
    sd.v64 = aos ? carve<double>(ws, L.v64) : nullptr;
    sd.flag = nullptr;
    // (slightly below (skin/2)^2, so rounding in the displacement can only
    // rebuild early)
    sd.disp2 = half_skin * half_skin * (1.0 - std::ldexp(1.0, -20));
    // With a skin, each step's force pass reads the rows of the pairs now
    // inside r_c, filtered out of the list (built at r_c + skin) in order:
    // the list entries between r_c and r_c + skin would otherwise take a
    // lane of the force pass each.
    ForceArgs af = a;
    int32_t* kept_off = skin ? carve<int32_t>(ws, L.kept_off) : nullptr;
    if (skin) {
        af.slab = carve<int32_t>(ws, L.kept);
        af.slab_flag = carve<int32_t>(ws, L.kept_flag);
        af.offset = kept_off;
        af.capacity = a.capacity;                        // kept rows are never longer than the list's
    }
    // Without a skin: each step's second half-kick (and the next step's
    // first half-kick and drift) runs in the force pass's row epilogue, which
    // has the row's force at hand; its statistics follow the force pass.  The
    // pass reads velocities only from the reorder's copies (FP32 in the mixed
    // form, the packed FP64 records in the FP64 form), never the state's v,
    // which the last step's epilogue rewrites.
    const bool fuse_vv = !skin && !job.bv.kps;
    for (int32_t k = 0; k < n_steps; ++k) {
        Job jk = job;
        int32_t* g = skin ? gates + (k & 1) : nullptr;
        jk.gate = g;
        DPD_TRY(mark(k, 0), "event");
        if (k == 0) {
            if (skin) DPD_TRY(launch_fill_i32(g, 1, 1, s), "rebuild flag");
            DPD_TRY(launch_vv1(kp, job.bv, n, st->x, st->v, st->f, st->tag, st->type, b.x, b.v, bvt, b.tag, b.type, s),
                    "vv1");
        } else if (fuse_vv) {
            // (the previous step's force pass did phase 2 and this phase 1)
        } else if (skin) {
            DPD_TRY(launch_fill_i32(g, 1, 0, s), "rebuild flag");
            sd.flag = g;
            DPD_TRY(launch_drift_skin(kp, n, sd, red_part, a.fred_part, force_grid(a), fsum_part, s), "vv2 + vv1");
            DPD_TRY(launch_reduce_final(n, red_part, kRedBlocks, fsum_part, kRedBlocks,
                                        d_reductions ? d_reductions + 8 * (int64_t)(k - 1) : nullptr, nullptr,
                                        d_step, d_status, s, gates + ((k - 1) & 1)), "reduce");
            DPD_TRY(launch_precopy(n, st->x, st->v, vt_sorted, st->tag, st->type, b.x, b.v, bvt, b.tag, b.type, s, g),
                    "pre-reorder copy");
        } else {
            DPD_TRY(launch_vv2(kp, n, st->v, st->f, red_part, a.fred_part, force_grid(a), fsum_part, s, &drift),
                    "vv2 + vv1");
            DPD_TRY(launch_reduce_final(n, red_part, kRedBlocks, fsum_part, kRedBlocks,
                                        d_reductions ? d_reductions + 8 * (int64_t)(k - 1) : nullptr, nullptr,
                                        d_step, d_status, s), "reduce");
        }
        DPD_TRY(mark(k, 1), "event");
        rc = enqueue_reorder(jk, L, ws, &b, bvt, st, vt_sorted, cells, x32, mixed ? v32 : nullptr, s, aos,
                             k > 0 ? inv : nullptr, !bonds || skin || k == 0 || k == n_steps - 1);
        if (rc) return rc;
        if (bonds) {
            if (k == 0) {
                DPD_TRY(launch_pidx_init(kp, n, st->tag, cells->idx_of_tag, pidx_cur, s), "bond partners");
            } else {
                DPD_TRY(launch_pidx_update(n, cells->perm, inv, pidx_cur, pidx_nxt, s, g), "bond partners");
                std::swap(pidx_cur, pidx_nxt);
            }
            a.pidx = pidx_cur;
        }
        DPD_TRY(mark(k, 2), "event");
        // inside a call the force pass reads the builder's slab; the CSR list
        // is written for the last step, which the caller sees
        rc = enqueue_nlist(jk, L, ws, st, cells, x32, nl, d_status, s, k == n_steps - 1);
        if (rc) return rc;
        if (skin) {
            af.pidx = a.pidx;
            int32_t* kflag = carve<int32_t>(ws, L.kept_flag);
            DPD_TRY(launch_fill_i32(kflag, 1, 0, s), "kept rows flag");
            DPD_TRY(launch_skin_filter(kp, precision, a, carve<int32_t>(ws, L.kept), kept_off, kflag, s),
                    "rows inside r_c");
            DPD_TRY(launch_fill_i32(kept_off + n, 1, 0, s), "kept rows total");
            DPD_TRY(launch_scan(kept_off, (int64_t)n + 1, carve<int32_t>(ws, L.scan_part), s), "kept rows scan");
        }
        DPD_TRY(mark(k, 3), "event");
        if (fuse_vv) {
            ForceArgs av = a;
            av.vv_v = st->v;
            av.vv_part = red_part;
            // the last step stores v; the others drift into the reorder's source
            if (k < n_steps - 1) av.vv_drift = drift;
            DPD_TRY(launch_forces(kp, job.bv, precision, av, s), "forces + vv2");
            DPD_TRY(mark(k, 4), "event");
            DPD_TRY(launch_reduce_final(n, red_part, force_grid(a), a.fred_part, force_grid(a),
                                        d_reductions ? d_reductions + 8 * (int64_t)k : nullptr, nullptr, d_step,
                                        d_status, s, nullptr, force_grid(a)), "reduce");
            DPD_TRY(mark(k, 5), "event");
            continue;
        }
        DPD_TRY(launch_forces(kp, job.bv, precision, skin ? af : a, s), "forces");
        DPD_TRY(mark(k, 4), "event");
        if (k == n_steps - 1) {
            DPD_TRY(launch_vv2(kp, n, st->v, st->f, red_part, a.fred_part, force_grid(a), fsum_part, s), "vv2");
            DPD_TRY(launch_reduce_final(n, red_part, kRedBlocks, fsum_part, kRedBlocks,
                                        d_reductions ? d_reductions + 8 * (int64_t)k : nullptr, nullptr, d_step,
                                        d_status, s, g), "reduce");
        }
        DPD_TRY(mark(k, 5), "event");
    }
    return DPD_OK;
}

int dpd_forces_backward(const dpd_params* p, const dpd_state* sorted, const dpd_cells* cells,
                        const dpd_nlist* nl, uint64_t step, const double* grad_f, double* grad_x,
                        double* grad_v, double* grad_a, double* grad_gamma, int32_t accumulate, void* ws,
                        size_t ws_bytes, void* stream)
{
    KParams kp;
    int rc = make_kparams(p, &kp);
    if (rc) return rc;
    if ((rc = check_state(sorted, "sorted", false))) return rc;
    const int32_t n = sorted->n;
    if ((rc = check_nlist(nl, n))) return rc;
    const bool bonds = kp.partner != nullptr;
    if (bonds && (rc = check_cells(cells, n, true))) return rc;
    if (!grad_a || !grad_gamma) return fail(DPD_EINVAL, "grad_a / grad_gamma are NULL");
    if (n > 0 && (!grad_f || !grad_x || !grad_v)) return fail(DPD_EINVAL, "gradient arrays are NULL");
    const WsLayout L = ws_layout(kp, n);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    BackwardArgs a;
    a.n = n; a.x = sorted->x; a.v = sorted->v; a.tag = sorted->tag; a.type = sorted->type;
    a.offset = nl->offset; a.index = nl->index; a.capacity = nl->capacity;
    a.idx_of_tag = cells ? cells->idx_of_tag : nullptr;
    a.step = step; a.g = grad_f; a.xbar = grad_x; a.vbar = grad_v;
    a.part = carve<double>(ws, L.bwd_part);
    a.abar = grad_a; a.gbar = grad_gamma;
    a.acc_xv = accumulate ? 1 : 0;
    a.acc_params = accumulate ? 1 : 0;
    DPD_TRY(launch_forces_backward(kp, a, as_stream(stream)), "forces backward");
    return DPD_OK;
}

int dpd_step_backward(const dpd_params* p, const dpd_state* st, const dpd_cells* cells, const dpd_nlist* nl,
                      uint64_t step, const double* gx_in, const double* gv_in, const double* gf_in,
                      double* gx_out, double* gv_out, double* gf_out, double* grad_a, double* grad_gamma,
                      void* ws, size_t ws_bytes, void* stream)
{
    KParams kp;
    int rc = make_kparams(p, &kp);
    if (rc) return rc;
    if (!kp.lam_half) return fail(DPD_EUNSUPPORTED, "the step adjoint is implemented for lambda = 1/2");
    if ((rc = check_state(st, "state", true))) return rc;
    const int32_t n = st->n;
    if ((rc = check_nlist(nl, n)) || (rc = check_cells(cells, n, kp.partner != nullptr))) return rc;
    if (!grad_a || !grad_gamma) return fail(DPD_EINVAL, "grad_a / grad_gamma are NULL");
    if (n > 0 && (!gx_in || !gv_in || !gf_in || !gx_out || !gv_out || !gf_out))
        return fail(DPD_EINVAL, "adjoint arrays are NULL");
    if (n > 0 && (gx_out == gx_in || gv_out == gv_in || gf_out == gf_in))
        return fail(DPD_EINVAL, "adjoint outputs must not alias the inputs");
    const WsLayout L = ws_layout(kp, n);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    StepBackwardArgs b;
    BackwardArgs& a = b.fwd;
    a.n = n; a.x = st->x; a.v = nullptr; a.tag = st->tag; a.type = st->type;
    a.offset = nl->offset; a.index = nl->index; a.capacity = nl->capacity;
    a.idx_of_tag = cells->idx_of_tag;
    a.step = step; a.g = nullptr; a.xbar = nullptr; a.vbar = nullptr;
    a.part = carve<double>(ws, L.bwd_part);
    a.abar = grad_a; a.gbar = grad_gamma;
    a.acc_xv = 0; a.acc_params = 1;
    b.v_new = st->v; b.f_new = st->f; b.perm = cells->perm;
    b.gx_in = gx_in; b.gv_in = gv_in; b.gf_in = gf_in;
    b.gx_out = gx_out; b.gv_out = gv_out; b.gf_out = gf_out;
    // scratch: the pre-reorder buffers and the list slab are free here
    double* slab = carve<double>(ws, L.slab);
    b.vt = carve<double>(ws, L.bx);
    b.gf_eff = carve<double>(ws, L.bv);
    b.xphi = slab;
    b.vphi = slab + 3 * (size_t)(n > 0 ? n : 1);
    DPD_TRY(launch_step_backward(kp, b, as_stream(stream)), "step backward");
    return DPD_OK;
}

size_t dpd_border_workspace_bytes(int32_t n)
{
    if (n < 0) return 0;
    return border_ws_layout(n).total;
}

int dpd_border_lists(const dpd_state* st, const double lo[3], const double hi[3], double width, int32_t face_mask,
                     int32_t* send_offset, int32_t* send_index, int64_t capacity, int32_t* d_status, void* ws,
                     size_t ws_bytes, void* stream)
{
    if (!st) return fail(DPD_EINVAL, "state is NULL");
    if (st->n < 0) return fail(DPD_EINVAL, "state->n must be >= 0");
    if (st->n > 0 && !st->x) return fail(DPD_EINVAL, "state->x is NULL");
    if (!lo || !hi) return fail(DPD_EINVAL, "lo / hi is NULL");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(lo[d]) || !std::isfinite(hi[d]) || !(lo[d] < hi[d]))
            return fail(DPD_EINVAL, "brick must have finite lo[%d] < hi[%d]", d, d);
    if (!std::isfinite(width) || !(width >= 0.0)) return fail(DPD_EINVAL, "width must be finite and >= 0");
    if (face_mask < 0 || face_mask > 63) return fail(DPD_EINVAL, "face_mask must be in [0, 63]");
    if (!send_offset) return fail(DPD_EINVAL, "send_offset is NULL");
    if (capacity < 0 || capacity >= ((int64_t)1 << 31)) return fail(DPD_EINVAL, "capacity must be in [0, 2^31)");
    if (capacity > 0 && !send_index) return fail(DPD_EINVAL, "send_index is NULL");
    int rc;
    if ((rc = check_ws(ws, ws_bytes, border_ws_layout(st->n).total))) return rc;
    DPD_TRY(launch_border_lists(st->n, st->x, lo, hi, width, face_mask, send_offset, send_index, capacity, d_status,
                                ws, as_stream(stream)), "border lists");
    return DPD_OK;
}

int dpd_border_pack(const dpd_state* st, const int32_t* send_offset, const int32_t* send_index, int64_t capacity,
                    const double shift[18], dpd_ghost* records, int32_t* d_status, void* stream)
{
    int rc;
    if ((rc = check_state(st, "state", false))) return rc;
    if (!send_offset || !shift) return fail(DPD_EINVAL, "send_offset / shift is NULL");
    if (capacity < 0 || capacity >= ((int64_t)1 << 31)) return fail(DPD_EINVAL, "capacity must be in [0, 2^31)");
    if (capacity > 0 && (!send_index || !records)) return fail(DPD_EINVAL, "send_index / records is NULL");
    if (capacity > 0 && !aligned(records, 8)) return fail(DPD_EINVAL, "records must be 8-byte aligned");
    for (int q = 0; q < 18; ++q)
        if (!std::isfinite(shift[q])) return fail(DPD_EINVAL, "shift must be finite");
    if (capacity == 0) return DPD_OK;
    DPD_TRY(launch_border_pack(st->n, st->x, st->v, st->tag, st->type, send_offset, send_index, capacity, shift,
                               records, d_status, as_stream(stream)), "border pack");
    return DPD_OK;
}

int dpd_border_unpack(const dpd_ghost* records, const int32_t* d_count, int64_t capacity, dpd_state* dst,
                      int32_t first, int32_t* d_status, void* stream)
{
    int rc;
    if ((rc = check_state(dst, "dst", false))) return rc;
    if (!d_count) return fail(DPD_EINVAL, "d_count is NULL");
    if (capacity < 0 || capacity >= ((int64_t)1 << 31)) return fail(DPD_EINVAL, "capacity must be in [0, 2^31)");
    if (capacity > 0 && !records) return fail(DPD_EINVAL, "records is NULL");
    if (first < 0 || first > dst->n) return fail(DPD_EINVAL, "first must be in [0, dst->n]");
    if (capacity == 0) return DPD_OK;
    DPD_TRY(launch_border_unpack(records, d_count, capacity, dst->n, first, dst->x, dst->v, dst->tag, dst->type,
                                 d_status, as_stream(stream)), "border unpack");
    return DPD_OK;
}

int dpd_math_eval(int32_t fn, int64_t n, const double* a, const double* b, double* out, void* stream)
{
    if (fn < DPD_FN_LOG || fn > DPD_FN_FASTPOW) return fail(DPD_EINVAL, "unknown function %d", fn);
    if (n < 0) return fail(DPD_EINVAL, "n must be >= 0");
    if (n > 0 && (!a || !out)) return fail(DPD_EINVAL, "a / out is NULL");
    if (n > 0 && (fn == DPD_FN_POW || fn == DPD_FN_FASTPOW) && !b) return fail(DPD_EINVAL, "b is NULL");
    DPD_TRY(launch_numerics_eval(fn, n, a, (fn == DPD_FN_POW || fn == DPD_FN_FASTPOW) ? b : nullptr, out,
                                 as_stream(stream)), "math eval");
    return DPD_OK;
}

int dpd_math_latency(int32_t fn, int32_t chain, int64_t* d_cycles, double* d_sink, void* stream)
{
    if (fn < DPD_FN_LOG || fn > DPD_FN_FASTPOW) return fail(DPD_EINVAL, "unknown function %d", fn);
    if (chain < 1) return fail(DPD_EINVAL, "chain must be >= 1");
    if (!d_cycles || !d_sink) return fail(DPD_EINVAL, "d_cycles / d_sink is NULL");
    DPD_TRY(launch_numerics_latency(fn, chain, d_cycles, d_sink, as_stream(stream)), "math latency");
    return DPD_OK;
}

int dpd_tea_signatures(int32_t n, const uint32_t* tag, const double* v, uint64_t step, uint64_t seed,
                       uint32_t* sig, void* stream)
{
    if (n < 0) return fail(DPD_EINVAL, "n must be >= 0");
    if (n > 0 && (!tag || !v || !sig)) return fail(DPD_EINVAL, "tag / v / sig is NULL");
    DPD_TRY(launch_signatures(n, tag, v, step, seed, sig, as_stream(stream)), "signatures");
    return DPD_OK;
}

int dpd_tea_gaussians(int64_t n, const uint32_t* sig_i, const uint32_t* sig_j, uint64_t step, uint64_t seed,
                      uint32_t* words, double* xi, void* stream)
{
    if (n < 0) return fail(DPD_EINVAL, "n must be >= 0");
    if (n > 0 && (!sig_i || !sig_j || !xi)) return fail(DPD_EINVAL, "sig_i / sig_j / xi is NULL");
    DPD_TRY(launch_tea_gauss(n, sig_i, sig_j, step, seed, words, xi, as_stream(stream)), "TEA gaussians");
    return DPD_OK;
}

int dpd_gaussian_throughput(int32_t generator, int32_t n_tags, int32_t pairs_per_thread, uint64_t step,
                            uint64_t seed, const uint32_t* sig, double* sink, void* stream)
{
    if (generator != 0 && generator != 1) return fail(DPD_EINVAL, "generator must be 0 or 1");
    if (n_tags < 0 || pairs_per_thread < 0) return fail(DPD_EINVAL, "sizes must be >= 0");
    if (n_tags > 0 && (!sink || (generator == 1 && !sig))) return fail(DPD_EINVAL, "sink / sig is NULL");
    if (n_tags > 0 && pairs_per_thread >= n_tags)
        return fail(DPD_EINVAL, "pairs_per_thread must be below n_tags (a partner index wraps once)");
    DPD_TRY(launch_gauss_throughput(generator, n_tags, pairs_per_thread, step, seed, sig, sink, as_stream(stream)),
            "gaussian throughput");
    return DPD_OK;
}

size_t dpd_batch_table_bytes(int32_t n_sys, int64_t n_total)
{
    if (n_sys < 1 || n_sys > 65535 || n_total < n_sys || n_total >= ((int64_t)1 << 31)) return 0;
    return batch_table(n_sys, n_total).total;
}

int dpd_batch_create(const dpd_params* per_sys, int32_t n_sys, const int64_t* sys_offset, void* d_table,
                     size_t table_bytes, void* stream, dpd_batch** out)
{
    if (!out) return fail(DPD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!per_sys || !sys_offset) return fail(DPD_EINVAL, "per_sys / sys_offset is NULL");
    if (n_sys < 1 || n_sys > 65535) return fail(DPD_EINVAL, "n_sys must be in [1, 65535]");
    if (sys_offset[0] != 0) return fail(DPD_EINVAL, "sys_offset[0] must be 0");
    for (int32_t q = 0; q < n_sys; ++q)
        if (!(sys_offset[q + 1] > sys_offset[q]))
            return fail(DPD_EINVAL, "system %d is empty (sys_offset must increase strictly)", q);
    const int64_t n_total = sys_offset[n_sys];
    if (n_total >= ((int64_t)1 << 31)) return fail(DPD_EINVAL, "more than 2^31 - 1 particles");
    const BatchTable T = batch_table(n_sys, n_total);
    if (!d_table) return fail(DPD_EINVAL, "d_table is NULL");
    if (!aligned(d_table, 256)) return fail(DPD_EINVAL, "d_table must be 256-byte aligned");
    if (table_bytes < T.total) return fail(DPD_ECAPACITY, "d_table has %zu bytes, needs %zu", table_bytes, T.total);

    std::unique_ptr<dpd_batch> b(new dpd_batch());
    b->n_sys = n_sys;
    b->n_total = n_total;
    b->kps.resize(n_sys);
    b->p_off.resize(n_sys + 1);
    b->c_off.resize(n_sys + 1);
    b->b_off.resize(n_sys + 1);
    b->t_off.resize(n_sys + 1);
    b->ch_off.resize(n_sys + 1);
    const dpd_params& p0 = per_sys[0];
    int64_t c_tot = 0, b_tot = 0, t_tot = 0, ch_tot = 0;
    int32_t slab_k = 0;
    for (int32_t q = 0; q < n_sys; ++q) {
        const dpd_params& p = per_sys[q];
        if (p.bond_partner) return fail(DPD_EUNSUPPORTED, "system %d: bonds are not supported in a batch", q);
        if (p.r_c != p0.r_c || p.skin != p0.skin || p.dt != p0.dt || p.lambda != p0.lambda || p.s != p0.s ||
            p.n_types != p0.n_types)
            return fail(DPD_EUNSUPPORTED, "system %d differs from system 0 in r_c, skin, dt, lambda, s or n_types", q);
        KParams& k = b->kps[q];
        const int rc = make_kparams(&p, &k);
        if (rc) {
            const std::string why = g_error;
            return fail(rc, "system %d: %s", q, why.c_str());
        }
        const int32_t ns = (int32_t)(sys_offset[q + 1] - sys_offset[q]);
        k.p_off = (int32_t)sys_offset[q];
        k.c_off = (int32_t)c_tot;
        k.b_off = (int32_t)b_tot;
        k.t_off = (int32_t)t_tot;
        k.n_local = ns;
        b->p_off[q] = k.p_off;
        b->c_off[q] = k.c_off;
        b->b_off[q] = k.b_off;
        b->t_off[q] = k.t_off;
        b->ch_off[q] = (int32_t)ch_tot;
        ch_tot += (ns + kWave - 1) / kWave;
        c_tot += k.n_cells;
        b_tot += k.n_blocks;
        t_tot += k.n_tiles;
        if (c_tot >= ((int64_t)1 << 31) - 1 || b_tot >= ((int64_t)1 << 31) || t_tot >= ((int64_t)1 << 31))
            return fail(DPD_EINVAL, "too many cells");
        const double vol = k.L[0] * k.L[1] * k.L[2];
        const int32_t w = nlist_slab_width(ns / vol, k.rl2);
        slab_k = w > slab_k ? w : slab_k;
    }
    b->p_off[n_sys] = (int32_t)n_total;
    b->c_off[n_sys] = (int32_t)c_tot;
    b->b_off[n_sys] = (int32_t)b_tot;
    b->t_off[n_sys] = (int32_t)t_tot;
    b->ch_off[n_sys] = (int32_t)ch_tot;

    Job& job = b->job;
    job.kp = b->kps[0];
    job.kp.p_off = job.kp.c_off = job.kp.b_off = job.kp.t_off = 0;
    job.kp.n_local = 0;
    job.bv.kps = carve<KParams>(d_table, T.kps);
    job.bv.p_off = carve<int32_t>(d_table, T.p_off);
    job.bv.c_off = carve<int32_t>(d_table, T.c_off);
    job.bv.b_off = carve<int32_t>(d_table, T.b_off);
    job.bv.t_off = carve<int32_t>(d_table, T.t_off);
    job.bv.ch_off = carve<int32_t>(d_table, T.ch_off);
    job.bv.n_chunks = (int32_t)ch_tot;
    job.bv.sys_of = carve<uint16_t>(d_table, T.sys_of);
    job.bv.n_sys = n_sys;
    job.n_cells = (int32_t)c_tot;
    job.n_blocks = (int32_t)b_tot;
    job.n_tiles = (int32_t)t_tot;
    job.slab_k = slab_k;
    job.force_grid = 0;
    job.nlist_waves = 4;
    job.nlist_kind = 0;
    b->step_base = carve<uint64_t>(d_table, T.step_base);
    (void)force_blocks((int32_t)n_total, DPD_FP64);      // occupancy queries happen here, not under capture
    (void)force_blocks((int32_t)n_total, DPD_MIXED);

    const hipStream_t s = as_stream(stream);
    DPD_TRY(hipMemcpyAsync(carve<void>(d_table, T.kps), b->kps.data(), n_sys * sizeof(KParams),
                           hipMemcpyHostToDevice, s), "copy batch table");
    DPD_TRY(hipMemcpyAsync(carve<void>(d_table, T.p_off), b->p_off.data(), (n_sys + 1) * sizeof(int32_t),
                           hipMemcpyHostToDevice, s), "copy batch table");
    DPD_TRY(hipMemcpyAsync(carve<void>(d_table, T.c_off), b->c_off.data(), (n_sys + 1) * sizeof(int32_t),
                           hipMemcpyHostToDevice, s), "copy batch table");
    DPD_TRY(hipMemcpyAsync(carve<void>(d_table, T.b_off), b->b_off.data(), (n_sys + 1) * sizeof(int32_t),
                           hipMemcpyHostToDevice, s), "copy batch table");
    DPD_TRY(hipMemcpyAsync(carve<void>(d_table, T.t_off), b->t_off.data(), (n_sys + 1) * sizeof(int32_t),
                           hipMemcpyHostToDevice, s), "copy batch table");
    DPD_TRY(hipMemcpyAsync(carve<void>(d_table, T.ch_off), b->ch_off.data(), (n_sys + 1) * sizeof(int32_t),
                           hipMemcpyHostToDevice, s), "copy batch table");
    DPD_TRY(launch_sys_map(job.bv, (int32_t)n_total, carve<uint16_t>(d_table, T.sys_of), s), "system map");
    // the host vectors feed asynchronous copies: they must not move before
    // the copies have run, so the caller's stream is drained here
    DPD_TRY(hipStreamSynchronize(s), "batch setup");
    *out = b.release();
    return DPD_OK;
}

void dpd_batch_destroy(dpd_batch* b)
{
    if (!b) return;
    drop_graph(b);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    delete b;
}

int dpd_batch_sizes(const dpd_batch* b, int64_t* n_total, int64_t* n_cells_total)
{
    if (!b) return fail(DPD_EINVAL, "batch is NULL");
    if (n_total) *n_total = b->n_total;
    if (n_cells_total) *n_cells_total = b->job.n_cells;
    return DPD_OK;
}

size_t dpd_batch_workspace_bytes(const dpd_batch* b, int32_t precision)
{
    if (!b || (precision != DPD_FP64 && precision != DPD_MIXED)) return 0;
    return ws_layout(b->job, (int32_t)b->n_total, precision == DPD_FP64).total;
}

int dpd_batch_set_tiles(dpd_batch* b, const dpd_tiles* t)
{
    if (!b || !t) return fail(DPD_EINVAL, "NULL argument");
    if (t->force_grid != 0 && (t->force_grid < 64 || t->force_grid > kMaxForceGrid))
        return fail(DPD_EINVAL, "force_grid must be 0 or in [64, %d]", kMaxForceGrid);
    if (t->nlist_waves != 0 && t->nlist_waves != 1 && t->nlist_waves != 2 && t->nlist_waves != 4)
        return fail(DPD_EINVAL, "nlist_waves must be 0, 1, 2 or 4");
    if (t->nlist_kind < 0 || t->nlist_kind > 2) return fail(DPD_EINVAL, "nlist_kind must be 0, 1 or 2");
    if (t->reserved) return fail(DPD_EINVAL, "reserved field must be 0");
    const int32_t waves = t->nlist_waves ? t->nlist_waves : 4;
    if (t->force_grid != b->job.force_grid || waves != b->job.nlist_waves || t->nlist_kind != b->job.nlist_kind)
        drop_graph(b);
    b->job.force_grid = t->force_grid;
    b->job.nlist_waves = waves;
    b->job.nlist_kind = t->nlist_kind;
    return DPD_OK;
}

int dpd_batch_get_tiles(const dpd_batch* b, dpd_tiles* t)
{
    if (!b || !t) return fail(DPD_EINVAL, "NULL argument");
    std::memset(t, 0, sizeof(*t));
    t->force_grid = b->job.force_grid;
    t->nlist_waves = b->job.nlist_waves;
    t->nlist_kind = b->job.nlist_kind;
    return DPD_OK;
}

int dpd_batch_bin_reorder(const dpd_batch* b, const dpd_state* in, dpd_state* out, dpd_cells* cells,
                          float* x32, float* v32, void* ws, size_t ws_bytes, void* stream)
{
    if (!b) return fail(DPD_EINVAL, "batch is NULL");
    int rc;
    if ((rc = check_batch_state(b, in, "in", false)) || (rc = check_batch_state(b, out, "out", false))) return rc;
    if (in->x == out->x || in->v == out->v || in->tag == out->tag || in->type == out->type)
        return fail(DPD_EINVAL, "in and out must not overlap");
    if ((rc = check_cells(cells, in->n, false))) return rc;
    const WsLayout L = ws_layout(b->job, in->n);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    if ((rc = enqueue_rank_table(b->job, L, ws, as_stream(stream)))) return rc;
    return enqueue_reorder(b->job, L, ws, in, nullptr, out, nullptr, cells, x32, v32, as_stream(stream));
}

int dpd_batch_build_neighbors(const dpd_batch* b, const dpd_state* sorted, const dpd_cells* cells,
                              const float* x32, dpd_nlist* nl, int32_t* d_status, void* ws,
                              size_t ws_bytes, void* stream)
{
    if (!b) return fail(DPD_EINVAL, "batch is NULL");
    int rc;
    if (!sorted) return fail(DPD_EINVAL, "sorted is NULL");
    if ((int64_t)sorted->n != b->n_total) return fail(DPD_EINVAL, "sorted->n does not match the batch");
    if (!sorted->x) return fail(DPD_EINVAL, "sorted->x is NULL");
    if ((rc = check_cells(cells, sorted->n, false)) || (rc = check_nlist(nl, sorted->n))) return rc;
    if (!x32) return fail(DPD_EINVAL, "x32 (from dpd_batch_bin_reorder) is NULL");
    const WsLayout L = ws_layout(b->job, sorted->n);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    if ((rc = enqueue_rank_table(b->job, L, ws, as_stream(stream)))) return rc;
    return enqueue_nlist(b->job, L, ws, sorted, cells, x32, nl, d_status, as_stream(stream));
}

int dpd_batch_forces(const dpd_batch* b, int32_t precision, const dpd_state* sorted, const dpd_cells* cells,
                     const float* x32, const float* v32, const dpd_nlist* nl, uint64_t step,
                     double* f_out, double* pe_out, int32_t* d_status, void* ws, size_t ws_bytes,
                     void* stream)
{
    if (!b) return fail(DPD_EINVAL, "batch is NULL");
    if (precision != DPD_FP64 && precision != DPD_MIXED) return fail(DPD_EINVAL, "unknown precision %d", precision);
    int rc;
    if ((rc = check_batch_state(b, sorted, "sorted", false))) return rc;
    const int32_t n = sorted->n;
    if ((rc = check_nlist(nl, n))) return rc;
    if (!f_out) return fail(DPD_EINVAL, "f_out is NULL");
    if (precision == DPD_MIXED && (!x32 || !v32)) return fail(DPD_EINVAL, "mixed precision needs x32 and v32");
    if (precision == DPD_MIXED && (!aligned(x32, 16) || !aligned(v32, 16)))
        return fail(DPD_EINVAL, "x32 / v32 must be 16-byte aligned");
    const WsLayout L = ws_layout(b->job, n);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    ForceArgs a;
    a.n = n; a.x = sorted->x; a.v = sorted->v; a.tag = sorted->tag; a.type = sorted->type;
    a.cell_xyz = cells ? cells->cell_xyz : nullptr; a.x32 = x32; a.v32 = v32;
    a.offset = nl->offset; a.index = nl->index; a.capacity = nl->capacity;
    a.idx_of_tag = cells ? cells->idx_of_tag : nullptr;
    a.d_step = nullptr; a.step_add = step;
    a.f = f_out; a.pe = pe_out; a.npair = nullptr; a.fred_part = nullptr;
    a.status = d_status;
    a.grid = b->job.force_grid > 0 ? b->job.force_grid : force_blocks(n, precision);
    a.slab = nullptr; a.slab_k = 0; a.slab_flag = nullptr; a.slab_coded = 0;
    a.x64 = nullptr; a.v64 = nullptr;
    DPD_TRY(launch_forces(b->job.kp, b->job.bv, precision, a, as_stream(stream)), "forces");
    return DPD_OK;
}

int dpd_batch_step(dpd_batch* b, int32_t precision, dpd_state* st, int32_t n_steps, uint64_t* d_step,
                   double* d_reductions, dpd_cells* cells, dpd_nlist* nl, float* x32, float* v32,
                   int32_t* d_status, int32_t use_graph, void* ws, size_t ws_bytes, void* stream)
{
    if (!b) return fail(DPD_EINVAL, "batch is NULL");
    if (precision != DPD_FP64 && precision != DPD_MIXED) return fail(DPD_EINVAL, "unknown precision %d", precision);
    int rc;
    if ((rc = check_batch_state(b, st, "state", true))) return rc;
    if (n_steps < 0) return fail(DPD_EINVAL, "n_steps must be >= 0");
    if (!d_step) return fail(DPD_EINVAL, "d_step is NULL");
    const int32_t n = st->n;
    if ((rc = check_cells(cells, n, false)) || (rc = check_nlist(nl, n))) return rc;
    if (!x32) return fail(DPD_EINVAL, "x32 is NULL (the list build needs it)");
    if (precision == DPD_MIXED && !v32) return fail(DPD_EINVAL, "mixed precision needs v32");
    const WsLayout L = ws_layout(b->job, n, precision == DPD_FP64);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    if (n_steps == 0) return DPD_OK;
    const hipStream_t s = as_stream(stream);
    if ((rc = enqueue_rank_table(b->job, L, ws, s))) return rc;
    DPD_TRY(launch_counter(b->step_base, d_step, s), "step base");
    // the steps' forces read the builder's slab; the CSR index of the last
    // step's list is written once, at the end
    auto compact = [&]() -> int {
        DPD_TRY(launch_nlist_compact(n, nl->offset, nl->capacity, carve<int32_t>(ws, L.slab), L.slab_k,
                                     carve<int32_t>(ws, L.slab_flag), nl->index, s), "neighbour list");
        return DPD_OK;
    };
    if (!use_graph) {
        for (int32_t k = 0; k < n_steps; ++k)
            if ((rc = enqueue_batch_step(b, L, ws, precision, st, d_step, d_reductions, cells, nl, x32, v32,
                                         d_status, s)))
                return rc;
        return compact();
    }
    GraphKey key;
    std::memset(&key, 0, sizeof(key));
    key.precision = precision;
    key.force_grid = b->job.force_grid;
    key.nlist_waves = b->job.nlist_waves;
    key.nlist_kind = b->job.nlist_kind;
    key.pairs_once = pair_mode();
    key.st = *st; key.cells = *cells; key.nl = *nl;
    key.d_step = d_step; key.red = d_reductions; key.x32 = x32; key.v32 = v32; key.d_status = d_status;
    key.ws = ws; key.ws_bytes = ws_bytes;
    if (!b->exec || !b->have_key || std::memcmp(&key, &b->key, sizeof(key)) != 0) {
        drop_graph(b);
        if (!b->capture) DPD_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking), "capture stream");
        DPD_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal), "begin capture");
        rc = enqueue_batch_step(b, L, ws, precision, st, d_step, d_reductions, cells, nl, x32, v32, d_status,
                                b->capture);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->capture, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return hip_fail(ei, "instantiate graph");
        b->exec = exec;
        b->key = key;
        b->have_key = true;
    }
    for (int32_t k = 0; k < n_steps; ++k) DPD_TRY(hipGraphLaunch(b->exec, s), "graph launch");
    return compact();
}

}  // extern "C"
