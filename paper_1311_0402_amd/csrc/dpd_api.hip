// dpd_api.hip -- the C ABI of libdpd (declared in include/dpd.h).
//
// Host-side work only: argument validation, derived parameters, workspace
// carving and the order in which the kernels of one time step are enqueued.
// No entry point synchronises, allocates device memory or throws.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

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
    k->rl2 = r_list * r_list;
    // FP32 separations from cell offsets are within ~3e-6 r_list^2 of the
    // FP64 value (offsets below 4 cells); the band is ten times wider
    k->list_lo32 = (float)(k->rl2 * (1.0 - std::ldexp(1.0, -15)));
    k->list_hi32 = (float)(k->rl2 * (1.0 + std::ldexp(1.0, -15)));
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

WsLayout ws_layout(int32_t n, int32_t n_cells, bool need_vt, int32_t n_types)
{
    WsLayout w;
    size_t o = 0;
    const size_t N = (size_t)(n > 0 ? n : 1);
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
    const int64_t scan_items = (int64_t)(n > n_cells ? n : n_cells) + 1;
    w.scan_part = take((size_t)ceil_div(scan_items, kScanTile) * sizeof(int32_t) + 64);
    w.rank_tab = take((size_t)(n_cells > 0 ? n_cells : 1) * sizeof(int32_t));
    w.red_part = take((size_t)3 * kRedBlocks * 2 * sizeof(double));
    w.fred_part = take((size_t)force_blocks(n) * 2 * sizeof(double));
    w.bwd_part = take((size_t)backward_part_doubles(n, n_types) * sizeof(double));
    w.total = o;
    return w;
}

namespace {

// binning + reordering from `in` into `out` (shared by dpd_bin_reorder and dpd_step)
int enqueue_reorder(const KParams& kp, const WsLayout& L, void* ws, const dpd_state* in,
                    const double* vt_in, dpd_state* out, double* vt_out, dpd_cells* cells,
                    float* x32, float* v32, hipStream_t s)
{
    const int32_t n = in->n;
    int32_t* key = carve<int32_t>(ws, L.key);
    int32_t* slot = carve<int32_t>(ws, L.slot);
    uint32_t* cxyz = carve<uint32_t>(ws, L.cxyz);
    uint32_t* tmp_tag = carve<uint32_t>(ws, L.tmp_tag);
    int32_t* tmp_src = carve<int32_t>(ws, L.tmp_src);
    int32_t* part = carve<int32_t>(ws, L.scan_part);
    const int32_t* rank_tab = carve<int32_t>(ws, L.rank_tab);
    DPD_TRY(launch_fill_i32(cells->cell_start, (int64_t)kp.n_cells + 1, 0, s), "fill cell counts");
    DPD_TRY(launch_bin(kp, n, in->x, rank_tab, key, slot, cxyz, cells->cell_start, s), "bin");
    DPD_TRY(launch_scan(cells->cell_start, (int64_t)kp.n_cells + 1, part, s), "scan cells");
    DPD_TRY(launch_place(n, key, slot, cells->cell_start, in->tag, tmp_tag, tmp_src, s), "place");
    GatherArgs g;
    g.x_in = in->x; g.v_in = in->v; g.vt_in = vt_in; g.type_in = in->type; g.cxyz_in = cxyz;
    g.x_out = out->x; g.v_out = out->v; g.vt_out = vt_out; g.tag_out = out->tag; g.type_out = out->type;
    g.cell_xyz = cells->cell_xyz; g.perm = cells->perm; g.idx_of_tag = cells->idx_of_tag;
    g.x32 = x32; g.v32 = v32;
    DPD_TRY(launch_finalize(kp, n, key, cells->cell_start, tmp_tag, tmp_src, g, s), "finalize");
    return DPD_OK;
}

int enqueue_nlist(const KParams& kp, const WsLayout& L, void* ws, const dpd_state* st,
                  const dpd_cells* cells, const float* x32, dpd_nlist* nl, int32_t* d_status, hipStream_t s)
{
    const int32_t n = st->n;
    int32_t* part = carve<int32_t>(ws, L.scan_part);
    const int32_t* rank_tab = carve<int32_t>(ws, L.rank_tab);
    DPD_TRY(launch_fill_i32(nl->offset + n, 1, 0, s), "clear offset tail");
    DPD_TRY(launch_nlist_count(kp, n, st->x, x32, cells->cell_xyz, cells->cell_start, rank_tab, nl->offset, s),
            "nlist count");
    DPD_TRY(launch_scan(nl->offset, (int64_t)n + 1, part, s), "scan rows");
    DPD_TRY(launch_nlist_check(n, nl->offset, nl->capacity, d_status, s), "nlist check");
    DPD_TRY(launch_nlist_fill(kp, n, st->x, x32, cells->cell_xyz, cells->cell_start, rank_tab, nl->offset,
                              nl->index, nl->capacity, s), "nlist fill");
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

}  // namespace
}  // namespace dpd

using namespace dpd;

extern "C" {

const char* dpd_last_error(void) { return g_error.c_str(); }

const char* dpd_version(void) { return "libdpd 0.1 (gfx950)"; }

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
    return ws_layout(n, k.n_cells, !k.lam_half, k.n_types).total;
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
    const WsLayout L = ws_layout(in->n, kp.n_cells, !kp.lam_half, kp.n_types);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    DPD_TRY(launch_rank_table(kp, carve<int32_t>(ws, L.rank_tab), as_stream(stream)), "rank table");
    return enqueue_reorder(kp, L, ws, in, nullptr, out, nullptr, cells, x32, v32, as_stream(stream));
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
    const WsLayout L = ws_layout(sorted->n, kp.n_cells, !kp.lam_half, kp.n_types);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    DPD_TRY(launch_rank_table(kp, carve<int32_t>(ws, L.rank_tab), as_stream(stream)), "rank table");
    return enqueue_nlist(kp, L, ws, sorted, cells, x32, nl, d_status, as_stream(stream));
}

int dpd_forces(const dpd_params* p, int32_t precision, const dpd_state* sorted, const dpd_cells* cells,
               const float* x32, const float* v32, const dpd_nlist* nl, uint64_t step, double* f_out,
               double* pe_out, double* stats, int32_t* d_status, void* ws, size_t ws_bytes, void* stream)
{
    KParams kp;
    int rc = make_kparams(p, &kp);
    if (rc) return rc;
    if (precision != DPD_FP64 && precision != DPD_MIXED) return fail(DPD_EINVAL, "unknown precision %d", precision);
    if ((rc = check_state(sorted, "sorted", false))) return rc;
    const int32_t n = sorted->n;
    if ((rc = check_nlist(nl, n))) return rc;
    if (n > 0 && !f_out) return fail(DPD_EINVAL, "f_out is NULL");
    const bool bonds = kp.partner != nullptr;
    if (bonds || precision == DPD_MIXED) {
        if ((rc = check_cells(cells, n, bonds))) return rc;
    }
    if (precision == DPD_MIXED && n > 0 && (!x32 || !v32))
        return fail(DPD_EINVAL, "mixed precision needs x32 and v32");
    const WsLayout L = ws_layout(n, kp.n_cells, !kp.lam_half, kp.n_types);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    const hipStream_t s = as_stream(stream);
    ForceArgs a;
    a.n = n; a.x = sorted->x; a.v = sorted->v; a.tag = sorted->tag; a.type = sorted->type;
    a.cell_xyz = cells ? cells->cell_xyz : nullptr; a.x32 = x32; a.v32 = v32;
    a.offset = nl->offset; a.index = nl->index; a.capacity = nl->capacity;
    a.idx_of_tag = cells ? cells->idx_of_tag : nullptr;
    a.d_step = nullptr; a.step_add = step;
    a.f = f_out; a.pe = pe_out;
    a.fred_part = stats ? carve<double>(ws, L.fred_part) : nullptr;
    a.status = d_status;
    DPD_TRY(launch_forces(kp, precision, a, s), "forces");
    if (stats)
        DPD_TRY(launch_reduce_final(n, nullptr, 0, a.fred_part, force_blocks(n), nullptr, stats, nullptr,
                                    d_status, s), "force stats");
    return DPD_OK;
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
    const WsLayout L = ws_layout(n, kp.n_cells, !kp.lam_half, kp.n_types);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    if (n == 0 || n_steps == 0) return DPD_OK;
    const hipStream_t s = as_stream(stream);
    DPD_TRY(launch_rank_table(kp, carve<int32_t>(ws, L.rank_tab), s), "rank table");

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
    a.f = st->f; a.pe = nullptr;
    a.fred_part = carve<double>(ws, L.fred_part);
    a.status = d_status;
    double* red_part = carve<double>(ws, L.red_part);
    const bool mixed = precision == DPD_MIXED;

    auto mark = [&](int32_t k, int phase) -> hipError_t {
        if (!phase_events) return hipSuccess;
        return hipEventRecord(reinterpret_cast<hipEvent_t>(phase_events[6 * (int64_t)k + phase]), s);
    };
    for (int32_t k = 0; k < n_steps; ++k) {
        DPD_TRY(mark(k, 0), "event");
        DPD_TRY(launch_vv1(kp, n, st->x, st->v, st->f, st->tag, st->type, b.x, b.v, bvt, b.tag, b.type, s), "vv1");
        DPD_TRY(mark(k, 1), "event");
        rc = enqueue_reorder(kp, L, ws, &b, bvt, st, vt_sorted, cells, x32, mixed ? v32 : nullptr, s);
        if (rc) return rc;
        DPD_TRY(mark(k, 2), "event");
        rc = enqueue_nlist(kp, L, ws, st, cells, x32, nl, d_status, s);
        if (rc) return rc;
        DPD_TRY(mark(k, 3), "event");
        DPD_TRY(launch_forces(kp, precision, a, s), "forces");
        DPD_TRY(mark(k, 4), "event");
        DPD_TRY(launch_vv2(kp, n, st->v, st->f, red_part, s), "vv2");
        DPD_TRY(launch_reduce_final(n, red_part, kRedBlocks, a.fred_part, force_blocks(n),
                                    d_reductions ? d_reductions + 8 * (int64_t)k : nullptr, nullptr, d_step,
                                    d_status, s), "reduce");
        DPD_TRY(mark(k, 5), "event");
    }
    return DPD_OK;
}

int dpd_forces_backward(const dpd_params* p, const dpd_state* sorted, const dpd_cells* cells,
                        const dpd_nlist* nl, uint64_t step, const double* grad_f, double* grad_x,
                        double* grad_v, double* grad_a, double* grad_gamma, void* ws, size_t ws_bytes,
                        void* stream)
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
    const WsLayout L = ws_layout(n, kp.n_cells, !kp.lam_half, kp.n_types);
    if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
    BackwardArgs a;
    a.n = n; a.x = sorted->x; a.v = sorted->v; a.tag = sorted->tag; a.type = sorted->type;
    a.offset = nl->offset; a.index = nl->index; a.capacity = nl->capacity;
    a.idx_of_tag = cells ? cells->idx_of_tag : nullptr;
    a.step = step; a.g = grad_f; a.xbar = grad_x; a.vbar = grad_v;
    a.part = carve<double>(ws, L.bwd_part);
    a.abar = grad_a; a.gbar = grad_gamma;
    DPD_TRY(launch_forces_backward(kp, a, as_stream(stream)), "forces backward");
    return DPD_OK;
}

}  // extern "C"
