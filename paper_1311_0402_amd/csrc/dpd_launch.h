// dpd_launch.h -- host-side launchers of the DPD kernels (internal to libdpd).
//
// Each launcher enqueues its kernel(s) on `stream` and returns the launch
// status; none of them synchronises or allocates.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "dpd.h"
#include "dpd_common.h"

namespace dpd {

constexpr int kBlock = 256;          // threads per block for element-wise kernels
constexpr int kScanTile = 4096;      // items per block of the device-wide scan
constexpr int kRedBlocks = 1024;     // fixed grid of the velocity reductions

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ---- workspace layout (one workspace serves every entry point) ----
struct WsLayout {
    size_t bx, bv, bvt, btag, btype;   // post-drift, pre-reorder state (step)
    size_t vt_sorted;                  // reordered predicted velocity (lambda != 1/2)
    size_t key, slot, cxyz;            // binning: cell rank, slot in cell, cell coords
    size_t tmp_tag, tmp_src, tmp_key;  // scatter before the in-cell tag order
    size_t scan_part;                  // partial sums of the device-wide scan
    size_t rank_tab;                   // Morton rank of every cell (row-major cell index)
    size_t slab;                       // neighbour rows before compaction, K slots per particle
    size_t slab_flag;                  // set when some row did not fit its K slots
    int32_t slab_k;
    size_t red_part;                   // velocity reduction partials
    size_t fred_part;                  // force-kernel partials (PE, pairs)
    size_t fsum_part;                  // force partials folded to kRedBlocks columns
    size_t bwd_part;                   // adjoint partials (type-pair matrices)
    size_t pe_part;                    // per-particle potential energy (batch statistics)
    size_t x64, v64;                   // packed FP64 copies for the FP64 step (0 when not laid out)
    size_t np_part;                    // per-particle pair count (batch statistics)
    size_t sys_part;                   // per-chunk sums of a batch's statistics (6 per chunk)
    size_t tile_rest;                  // tiles left by the tile list builder: count, then tile ids
    size_t pidx_a, pidx_b, inv;        // bonds inside a step loop: partner indices (2 per particle,
                                       // two generations) and the old -> new index map
    size_t xref;                       // skin > 0: positions at the last rebuild (sorted order)
    size_t gate;                       // skin > 0: two rebuild flags (steps alternate between them)
    size_t kept, kept_off, kept_flag;  // skin > 0: each step's rows inside r_c (slab layout), their
                                       // offsets (n + 1) and a zero slab flag
    size_t total;
};

WsLayout ws_layout(const KParams& kp, int32_t n, bool aos = false);

// ---- reorder (k_reorder.hip) ----
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t value, hipStream_t s, Gate gate = nullptr);
// three single words set to zero by one launch (null pointers skipped)
hipError_t launch_zero3(int32_t* a, int32_t* b, int32_t* c, hipStream_t s, Gate gate = nullptr);
// rank_tab[c_off + cx + nc_x (cy + nc_y cz)] = c_off + Morton rank of the cell
// (bv.kps == nullptr: one system, c_off = 0, c_tot = its cell count)
hipError_t launch_rank_table(const KParams& kp, const BatchView& bv, int32_t c_tot, int32_t* rank_tab,
                             hipStream_t s);
hipError_t launch_bin(const KParams& kp, const BatchView& bv, int32_t n, const double* x, const int32_t* rank_tab,
                      int32_t* key, int32_t* slot, uint32_t* cxyz, int32_t* counts, hipStream_t s,
                      Gate gate = nullptr);
// in-place exclusive scan of data[0 .. count); partials needs ceil(count/kScanTile) ints
hipError_t launch_scan(int32_t* data, int64_t count, int32_t* partials, hipStream_t s, Gate gate = nullptr);
hipError_t launch_place(int32_t n, const int32_t* key, const int32_t* slot, const int32_t* cell_start,
                        const uint32_t* tag, uint32_t* tmp_tag, int32_t* tmp_src, int32_t* tmp_key, hipStream_t s,
                        Gate gate = nullptr);
struct GatherArgs {
    const double* x_in; const double* v_in; const double* vt_in; const uint8_t* type_in;
    const uint32_t* cxyz_in;
    double* x_out; double* v_out; double* vt_out; uint32_t* tag_out; uint8_t* type_out;
    uint32_t* cell_xyz; int32_t* perm; int32_t* idx_of_tag;   // idx_of_tag nullable
    int32_t* inv = nullptr;         // nullable: inv[source index] = sorted index
    float* x32; float* v32;
    double* x64; double* v64;       // nullable: packed FP64 copies, double4 per particle
    double* xref = nullptr;         // nullable: a second copy of the sorted positions ([3][n])
};
// bond partners of the sorted particles as sorted indices: pidx[2 i + b] =
// idx_of_tag[partner[2 tag[i] + b]], -1 without a partner, -2 when the
// partner tag has no particle
hipError_t launch_pidx_init(const KParams& kp, int32_t n, const uint32_t* tag, const int32_t* idx_of_tag,
                            int32_t* pidx, hipStream_t s);
// after a reorder: pidx_new[2 d + b] = inv[pidx_old[2 perm[d] + b]] (negative values kept);
// a step that did not reorder (gate off) copies pidx_old
hipError_t launch_pidx_update(int32_t n, const int32_t* perm, const int32_t* inv, const int32_t* pidx_old,
                              int32_t* pidx_new, hipStream_t s, Gate gate = nullptr);
hipError_t launch_finalize(const KParams& kp, const BatchView& bv, int32_t n, const int32_t* tmp_key,
                           const int32_t* cell_start, const uint32_t* tmp_tag, const int32_t* tmp_src,
                           const GatherArgs& g, hipStream_t s, Gate gate = nullptr);
// (gated) copy of a sorted state into the reorder's source buffers: x, v
// ([3][n]), vt (nullable), tag, type
hipError_t launch_precopy(int32_t n, const double* x, const double* v, const double* vt, const uint32_t* tag,
                          const uint8_t* type, double* bx, double* bv, double* bvt, uint32_t* btag,
                          uint8_t* btype, hipStream_t s, Gate gate);

// ---- neighbour list (k_nlist.hip) ----
int32_t nlist_slab_width(double density, double rl2);
// Slab entries of the lane builder, when n < 2^26: bits 0..25 hold j, bits
// 26..31 the offset of j's cell from i's cell, (dx+1) | (dy+1) << 2 |
// (dz+1) << 4, so the mixed force pass needs no cell arithmetic.
constexpr int kSlabCodeShift = 26;
constexpr int32_t kSlabJMask = (1 << kSlabCodeShift) - 1;

// whole list build: row sizes + slab rows, scan, capacity check, compaction
// (or the direct pass when a row overflowed its slab row); n_blocks counts
// the 2x2x2 cell blocks of all systems, n_tiles their list-build tiles.
// kind 0: tile builder, 1: block builder, 2: lane builder (0 and 2 need
// cell_xyz and fewer than 2^27 cells, else the block builder runs); waves
// sizes the workgroups of builders 1 and 2; tile_rest (n_tiles + 1 ints)
// lists the tiles the tile builder leaves to the lane builder.
hipError_t launch_nlist(const KParams& kp, const BatchView& bv, int32_t n_cells, int32_t n_blocks, int32_t n_tiles,
                        int32_t n, const double* x, const float* x32, const uint32_t* cell_xyz,
                        const int32_t* cell_start, const int32_t* rank_tab, int32_t* offset, int32_t* index,
                        int64_t capacity, int32_t* slab, int32_t slab_k, int32_t* flag, int32_t* tile_rest,
                        int32_t* status, int32_t* scan_part, int waves, int kind, bool compact, hipStream_t s,
                        Gate gate = nullptr);
// whether that build leaves coded slab entries (tile and lane builders, n < 2^26)
bool nlist_slab_coded(int kind, const uint32_t* cell_xyz, int32_t n_cells, int32_t n);
// waves per workgroup of the tile builder for n particles in n_cells cells
int nlist_tile_waves(int32_t n, int32_t n_cells);
// the CSR index from the builder's slab rows (nothing while the slab flag
// is set: the direct pass wrote the rows then)
hipError_t launch_nlist_compact(int32_t n, const int32_t* offset, int64_t capacity, const int32_t* slab,
                                int32_t slab_k, const int32_t* flag, int32_t* index, hipStream_t s);
hipError_t launch_nlist_check(int32_t n, const int32_t* offset, int64_t capacity, int32_t* status,
                              hipStream_t s);

// ---- forces (k_force.hip) ----
// the next step's phase 1 fused after phase 2: bx, bv (, bvt) from x and
// the phase-2 velocity, and btag / btype copied (the outputs of launch_vv1)
struct DriftArgs {
    const double* x; const uint32_t* tag; const uint8_t* type;
    double* bx; double* bv; double* bvt; uint32_t* btag; uint8_t* btype;
};
struct ForceArgs {
    int32_t n;
    const double* x; const double* v; const uint32_t* tag; const uint8_t* type;
    const uint32_t* cell_xyz; const float* x32; const float* v32;
    const int32_t* offset; const int32_t* index; int64_t capacity;
    const int32_t* idx_of_tag;
    const int32_t* pidx = nullptr;                // nullable: bond partners' sorted indices, 2 per particle
                                                  //   (-1 none, -2 missing); else partner + idx_of_tag
    const uint64_t* d_step; uint64_t step_add;   // step = (d_step ? *d_step : 0) + step_add
    double* f; double* pe;                        // pe nullable
    int32_t* npair;                               // nullable: pairs inside r_c per particle
    double* fred_part;                            // [grid][2]: PE, pair count
    int32_t* status;                              // nullable
    int32_t grid;                                 // persistent workgroups (> 0)
    const int32_t* slab;                          // nullable: the list builder's slab (rows at i * slab_k),
    int32_t slab_k;                               //   read instead of index while *slab_flag == 0
    const int32_t* slab_flag;
    int32_t slab_coded;                           // slab entries carry the stencil offset (see below)
    const double* x64;                            // nullable: (x, y, z, tag bits) per sorted particle
    const double* v64;                            //   and (v~, type bits), double4 each (FP64 pass)
    int32_t pairs_once = -1;                      // pairs of one 64-row chunk evaluated once
                                                  //   (1), every entry (0), the pair mode's choice (-1)
    // Single systems only (nullable): the step's second half-kick in the
    // force pass's row epilogue, v = fma(dt/2, F, v_h) with v_h read from
    // vv_v, as launch_vv2 computes it; with vv_drift.bx the next step's
    // phase 1 follows (bx, bv, bvt, btag, btype), else v is stored back into
    // vv_v.  Momentum and |v|^2 partials go to vv_part[3][grid][2] (reduce
    // with red_stride = grid).  Nothing else in the pass may read vv_v.
    double* vv_v = nullptr;
    double* vv_part = nullptr;
    DriftArgs vv_drift{};
};
hipError_t launch_forces(const KParams& kp, const BatchView& bv, int precision, const ForceArgs& a,
                         hipStream_t s);
// a list built at r_c + skin: for each row i of the builder's slab, the
// entries now inside r_c in order, at kept[i * a.slab_k], their number in
// count[i] (single system); when the slab overflowed, count[i] gets the CSR
// row size and *kept_flag is set (the force pass then reads the CSR list);
// *kept_flag must be 0 before the launch
hipError_t launch_skin_filter(const KParams& kp, int precision, const ForceArgs& a, int32_t* kept, int32_t* count,
                              int32_t* kept_flag, hipStream_t s);
constexpr int kMaxForceGrid = 8192;
// library default of ForceArgs::pairs_once for a precision (0 FP64, 1
// mixed) under the process-wide pair mode (0 every entry, 1 pairs once,
// 2 pairs once in the FP64 form; 2 unless changed); set returns the previous
// mode
bool pairs_once_default(int precision);
int set_pair_mode(int mode);
int pair_mode();
// default persistent grid of the force pass (the workgroups resident at once)
int force_blocks(int32_t n, int precision);
// the grid a launch uses: ForceArgs.grid, set by the caller (> 0)
inline int force_grid(const ForceArgs& a) { return a.grid; }

// ---- integration and reductions (k_integrate.hip) ----
hipError_t launch_vv1(const KParams& kp, const BatchView& bat, int32_t n, const double* x, const double* v,
                      const double* f, const uint32_t* tag, const uint8_t* type, double* bx, double* bv,
                      double* bvt, uint32_t* btag, uint8_t* btype, hipStream_t s);
// per-system statistics of a batch: v (momentum, |v|^2), the per-particle
// PE and pair counts summed per 64-particle chunk into part[n_chunks][6],
// then per system over its chunks (fixed orders), written to row
// (*d_step - *base) of red[rows][n_sys][8] (red nullable).  With f
// (nullable), the chunk pass first applies the second half-kick
// v = fma(half_dt, F, v) and stores v.
hipError_t launch_sys_reduce(const BatchView& bat, int32_t n, double* v, const double* f, double half_dt,
                             const double* pe, const int32_t* npair, double* part, double* red,
                             const uint64_t* d_step, const uint64_t* base, int32_t* status, hipStream_t s);
// *dst = *src, or *dst += 1 when src is null (device step counters)
hipError_t launch_counter(uint64_t* dst, const uint64_t* src, hipStream_t s);
// particle -> system map of a batch
hipError_t launch_sys_map(const BatchView& bat, int32_t n, uint16_t* sys_of, hipStream_t s);
// phase 2 + momentum / |v|^2 partials (f == nullptr: the partials of v as it
// is); also folds the force partials (fred_part, n_fred blocks) into
// fsum_part[kRedBlocks][2]; drift (nullable) adds the next step's phase 1,
// and then v itself is left as it was (the reorder writes v_h into the state)
hipError_t launch_vv2(const KParams& kp, int32_t n, double* v, const double* f, double* red_part,
                      const double* fred_part, int32_t n_fred, double* fsum_part, hipStream_t s,
                      const DriftArgs* drift = nullptr);
// The first phase of a step with a Verlet skin, in place on the sorted
// state (no reorder follows unless the gate says so): v~ / v_h and x from
// the previous step's v_h and F (its second phase v = v_h + dt/2 F is summed
// for the statistics, not stored), the packed copies of the new state (FP32
// offsets from each particle's cell at the last rebuild, FP64 copies), and
// *flag |= 1 when some particle is more than skin / 2 (disp2: the squared
// threshold) from its position at the last rebuild.  Momentum and |v|^2
// partials and the force partials' fold as launch_vv2.
struct SkinDriftArgs {
    double* x; double* v; double* vt;             // sorted state, in place (vt nullable)
    const double* f;
    const uint32_t* tag; const uint8_t* type; const uint32_t* cell_xyz;
    const double* xref;                            // positions at the last rebuild
    float* x32; float* v32;                        // nullable
    double* x64; double* v64;                      // nullable
    int32_t* flag;
    double disp2;
};
hipError_t launch_drift_skin(const KParams& kp, int32_t n, const SkinDriftArgs& d, double* red_part,
                             const double* fred_part, int32_t n_fred, double* fsum_part, hipStream_t s);
// sums the partials in a fixed order; red (nullable) gets the 8 step totals
// (the last one: 1 when the step rebuilt the lists, read from *rebuilt, or
// 1 when rebuilt is null); stats (nullable) gets (PE, pairs); increments
// *d_step when non-null
// (red_part[k] of component k starts at 2 k red_stride)
hipError_t launch_reduce_final(int32_t n, const double* red_part, int n_red, const double* fred_part,
                               int n_fred, double* red, double* stats, uint64_t* d_step,
                               int32_t* status, hipStream_t s, const int32_t* rebuilt = nullptr,
                               int red_stride = kRedBlocks);

// ---- border determination and ghosts (k_border.hip) ----
struct BorderWs {
    int32_t n_blk;                     // blocks of kBlock particles
    size_t flags;                      // uint8 face bits per particle
    size_t cnt;                        // int32 [6 n_blk + 1]: per-block counts, scanned in place
    size_t scan_part;                  // partials of the scan
    size_t total;
};
BorderWs border_ws_layout(int32_t n);
// send lists of the selected faces (face_mask bit f = 2 d + s) of the brick
// [lo, hi): flag, scan of the per-block counts, compaction; send_offset[7]
// gets the face offsets, send_index the ascending lists (nothing written
// past capacity; the status bit reports a short buffer)
hipError_t launch_border_lists(int32_t n, const double* x, const double lo[3], const double hi[3], double width,
                               int32_t face_mask, int32_t* send_offset, int32_t* send_index, int64_t capacity,
                               int32_t* status, void* ws, hipStream_t s);
// one record per send-list entry: position + shift[face], velocity, tag, type
hipError_t launch_border_pack(int32_t n, const double* x, const double* v, const uint32_t* tag, const uint8_t* type,
                              const int32_t* send_offset, const int32_t* send_index, int64_t capacity,
                              const double shift[18], dpd_ghost* out, int32_t* status, hipStream_t s);
// records [0, *d_count) into the state arrays at [first, first + count)
hipError_t launch_border_unpack(const dpd_ghost* in, const int32_t* d_count, int64_t capacity, int32_t n_dst,
                                int32_t first, double* x, double* v, uint32_t* tag, uint8_t* type, int32_t* status,
                                hipStream_t s);

// ---- the paper's numerics as A/B variants (k_numerics.hip) ----
hipError_t launch_numerics_eval(int fn, int64_t n, const double* a, const double* b, double* out, hipStream_t s);
hipError_t launch_numerics_latency(int fn, int32_t chain, int64_t* cycles, double* sink, hipStream_t s);
hipError_t launch_signatures(int32_t n, const uint32_t* tag, const double* v, uint64_t step, uint64_t seed,
                             uint32_t* sig, hipStream_t s);
hipError_t launch_tea_gauss(int64_t n, const uint32_t* si, const uint32_t* sj, uint64_t step, uint64_t seed,
                            uint32_t* w, double* xi, hipStream_t s);
hipError_t launch_gauss_throughput(int gen, int32_t n_tags, int32_t pairs_per_thread, uint64_t step, uint64_t seed,
                                   const uint32_t* sig, double* sink, hipStream_t s);

// ---- adjoint (k_adjoint.hip) ----
struct BackwardArgs {
    int32_t n;
    const double* x; const double* v; const uint32_t* tag; const uint8_t* type;
    const int32_t* offset; const int32_t* index; int64_t capacity;
    const int32_t* idx_of_tag;
    uint64_t step;
    const double* g;
    double* xbar; double* vbar;
    double* part;          // [blocks][2 * n_types^2]
    double* abar; double* gbar;
    int acc_xv;            // add into xbar / vbar instead of overwriting
    int acc_params;        // add into abar / gbar instead of overwriting
};
hipError_t launch_forces_backward(const KParams& kp, const BackwardArgs& a, hipStream_t s);

struct StepBackwardArgs {
    BackwardArgs fwd;      // state of the later step (x', tags, types, list); abar / gbar accumulate
    const double* v_new; const double* f_new;
    const int32_t* perm;
    const double* gx_in; const double* gv_in; const double* gf_in;
    double* gx_out; double* gv_out; double* gf_out;
    double* vt; double* gf_eff; double* xphi; double* vphi;   // workspace, [3][n] each
};
hipError_t launch_step_backward(const KParams& kp, const StepBackwardArgs& b, hipStream_t s);
int backward_part_doubles(int32_t n, int32_t n_types);

}  // namespace dpd
