// Fast multipole evaluation of the hybrid representation (App. E, Alg. 8)
// on the scene quadtree.  Host-side driver interface.
#pragma once

#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "dc_common.h"

struct dc_scene_s;

namespace dc {

// One viewport's target boxes at one level of a (batched) render.
struct VpLevel {
    long long i0, j0;      // rectangle of boxes at this level
    long long pi0, pj0;    // rectangle at the parent level
    int wl, pwl;           // rectangle widths
    int off, poff;         // global index of the first box, and of the parent's
    int first_block;       // first block of this viewport in the level's launch
    int hl;                // rectangle height
    int level, pad;        // quadtree level of the rectangle
};

// One viewport's target leaves (pixel tiles) in a (batched) render.
struct VpLeaf {
    long long i0, j0;
    double vcx, vcy, vw, vh;
    void* out;
    int L, wl, off, W, H, first_block;
    int hl, pad;             // tile rectangle height
    // offsets into the plan's edge table: pixel columns [E[col_at + i],
    // E[col_at + i + 1]) lie in tile column i0 + i; pixel rows
    // [E[row_at + j + 1], E[row_at + j]) in tile row j0 + j
    int col_at, row_at;
};

// Pinned host staging for descriptor uploads: reused once the copy that
// last read it has completed.
struct PinnedStage {
    void* p = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
    PinnedStage() = default;
    PinnedStage(const PinnedStage&) = delete;
    PinnedStage& operator=(const PinnedStage&) = delete;
    ~PinnedStage() {
        if (done) (void)hipEventSynchronize(done), (void)hipEventDestroy(done);
        if (p) (void)hipHostFree(p);
    }
    // Host pointer of at least nbytes, free for writing.
    void* acquire(size_t nbytes) {
        if (pending) DC_HIP(hipEventSynchronize(done));
        pending = false;
        if (nbytes > bytes) {
            if (p) DC_HIP(hipHostFree(p));
            p = nullptr;
            bytes = 0;
            DC_HIP(hipHostMalloc(&p, nbytes, hipHostMallocDefault));
            bytes = nbytes;
        }
        if (!done) DC_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
        return p;
    }
    // Mark the staging busy until the work queued so far on st has run.
    void mark_used(hipStream_t st) {
        DC_HIP(hipEventRecord(done, st));
        pending = true;
    }
};

// Host plan of one render of n viewports: per (viewport, level) rectangles
// of target boxes, launch sizes and the layout of the render's device
// scratch, [level table | leaf table | edge table | level index | local
// coefficients | near sets | expansion owners | done flags | claim counter |
// heavy-tile queue | kept traversal lists].
struct RenderPlan {
    int n = 0, p = 0, tile_px = 0, maxL = 0;
    std::vector<VpLevel> lev;
    std::vector<int> lev_begin, lev_blocks;
    std::vector<VpLeaf> leaf;
    std::vector<int> edges;  // pixel index ranges of tile columns and rows
    std::vector<int> vlev;   // [viewport][level] -> index into lev, or -1
    int leaf_blocks = 0;
    long long total_boxes = 0;
    size_t leaf_at = 0, edges_at = 0, vlev_at = 0, desc_bytes = 0, tl_at = 0, nset_at = 0;
    size_t owner_at = 0, scratch_bytes = 0;
    // per-box done flags and the claim counter of the persistent downward pass
    size_t done_at = 0, dctl_at = 0;
    // own incoming terms and quiet flags of the split downward pass
    size_t c_at = 0, quiet_at = 0;
    // queue of heavy small tiles (k_tile_scan, k_tile_big; 8-pixel tiles)
    size_t hv_ctl_at = 0, hv_list_at = 0, hv_flag_at = 0;
    // first-round traversal lists of light small tiles (k_tile_scan -> k_tile)
    size_t lists_at = 0;
    // Write both descriptor tables (desc_bytes) to host, with output
    // pointers outs[v].
    void write_tables(void* host, void* const* outs) const;
};

struct FmmState {
    // Quadtree on the device (copied from the host tree).
    int n_cells = 0, depth = 0, n_pieces = 0, n_target_leaves = 0;
    double X0 = 0, Y0 = 0, side = 1;
    std::vector<int> level_start;
    DevBuf<int> lvl, child, parent, pbeg, pend, npc, nbeg, nend, node_perm, target_leaves;
    DevBuf<int> cmask;  // per box: bit q set when child q holds pieces (0 for leaves)
    DevBuf<long long> ix, iy;
    // Pieces: start point, unit tangent, length, end point, segment.
    DevBuf<double> px0, py0, px1, py1, ptx, pty, plen;
    DevBuf<int> pseg;
    // Pieces of each segment (CSR), for the self-segment correction.
    DevBuf<int> seg_piece_beg, seg_piece_idx;
    // Piece weights (kappa sigma_bar, kappa mu_bar) [6][n_pieces].
    DevBuf<double> w64;
    DevBuf<float> w32;
    DevBuf<int> heavy;  // FP32 path: pieces evaluated in FP64
    // Multipole and local coefficients of the source tree (FP64 in both
    // precision modes), and near sets.
    DevBuf<double> M64, L64;
    DevBuf<double> Ms64;  // M64 with coefficient k divided by k (render M2P)
    // Tabulated incoming-from-outgoing operators per expansion order
    // (see m2l_table in fmm.hip).
    std::map<int, std::unique_ptr<DevBuf<double>>> m2l_tab;
    DevBuf<int> nsetS;
    // The solve's split downward pass: own incoming terms and quiet flags
    // of every cell.
    DevBuf<double> C64;
    DevBuf<unsigned char> quietS;
    // Cached near-field tables of the FP64 solve (SolveTables in fmm.hip),
    // built on the first FP64 operator application when they fit the budget.
    int tab_mode = 1;  // 0 off, 1 when they pay (dense near fields), 2 whenever they fit
    bool tab_tried = false, tab_ok = false;
    size_t tab_bytes = 0;
    long long tab_pairs = 0;
    DevBuf<long long> tab_pair_off;
    DevBuf<int> tab_piece_off, tab_w_off, tab_piece, tab_w;
    DevBuf<double> tab_val;
    // Cached P2M factors of order p2m_tab_p (k_p2m in fmm.hip), under the
    // same switch.
    DevBuf<double> p2m_tab;
    int p2m_tab_p = -1;
    // Upward pass of the resident densities (render reuses it); gen counts
    // the density changes (a captured render graph records it).
    bool up_valid = false;
    unsigned long long gen = 0;
    int up_p = -1, up_prec = -1;
    // Count of upward passes run (a captured render graph reads the
    // expansion buffers of one of them).
    unsigned long long up_epoch = 0;
    // Render of the dc_render / dc_render_batch calls: plan, descriptor
    // staging and device scratch (see RenderPlan).
    // The staging is a ring, so the host can plan the next render while the
    // device still runs the previous ones.
    RenderPlan plan;
    // Plan and host copy of the descriptor tables of dc_render_noalloc
    // (whose device scratch is a fixed array, see fmm.hip).
    RenderPlan noalloc_plan;
    std::vector<char> noalloc_tables;
    static constexpr int kStages = 3;
    PinnedStage stage[kStages];
    int stage_next = 0;
    DevBuf<char> scratch;
    // Optional device work counters (counting runs only) and phase timing.
    unsigned long long* stats = nullptr;
    bool timing = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    double tms[4] = {0, 0, 0, 0};
    int tcalls = 0;
    // Host word (pinned, mapped) that a render kernel sets when one of its
    // bounded waits ran out; reported and cleared by the scene's next call
    // that reaches fmm_check_stall.
    int* stall_host = nullptr;
    int* stall_dev = nullptr;
    // Second stream of the render leaf pass (queued heavy tiles run on it
    // concurrently with the other tiles), ordered by two events against
    // the caller's stream.  Renders of the scene on different caller
    // streams share it, which only serialises their heavy-tile kernels.
    // aux_mu is held from the stream's creation through the launch
    // sequence record(ev_scan) -> wait -> launches -> record(ev_big) ->
    // wait, so that a direct render and a server batch of the same scene
    // issued from two host threads cannot interleave their events.
    std::mutex aux_mu;
    hipStream_t aux = nullptr;
    hipEvent_t ev_scan = nullptr, ev_big = nullptr;
    hipStream_t aux_stream() {
        if (!aux) {
            DC_HIP(hipEventCreateWithFlags(&ev_scan, hipEventDisableTiming));
            DC_HIP(hipEventCreateWithFlags(&ev_big, hipEventDisableTiming));
            DC_HIP(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking));
        }
        return aux;
    }
    ~FmmState() {
        for (hipEvent_t& e : ev)
            if (e) (void)hipEventDestroy(e);
        if (aux) (void)hipStreamSynchronize(aux), (void)hipStreamDestroy(aux);
        if (ev_scan) (void)hipEventDestroy(ev_scan);
        if (ev_big) (void)hipEventDestroy(ev_big);
        if (stall_host) (void)hipHostFree(stall_host);
    }
};

std::unique_ptr<FmmState> fmm_create(const dc_scene_s& s);

// A render of fixed viewports and output buffers captured into a HIP
// graph (with its own plan, pinned descriptor tables and device scratch).
struct RenderGraph {
    dc_scene_s* s = nullptr;
    dc_eval_opts o{};
    int out_dtype = 0;
    unsigned long long gen = 0;
    unsigned long long up_epoch = 0;  // upward pass whose buffers the launches read
    RenderPlan plan;
    void* stage = nullptr;
    DevBuf<char> scratch;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    RenderGraph() = default;
    RenderGraph(const RenderGraph&) = delete;
    RenderGraph& operator=(const RenderGraph&) = delete;
    ~RenderGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (stage) (void)hipHostFree(stage);
    }
};
std::unique_ptr<RenderGraph> fmm_graph_create(dc_scene_s& s, const dc_viewport* vps, int n,
                                              const dc_eval_opts& o, int out_dtype,
                                              void* const* outs);
// Throws DC_ERR_INVALID when the scene's densities changed since the
// capture, or its resident expansions were rebuilt for another order or
// precision (their buffers may have moved: the graph must be made again).
void fmm_graph_launch(RenderGraph& g, hipStream_t st);
// Throws DC_ERR_TIMEOUT (and clears the word) when an earlier render of the
// scene stalled on the device; its images are then incomplete.
void fmm_check_stall(FmmState& f);
void fmm_invalidate(FmmState& f);
// y[3][N] = G_H sigma + F_H mu at the nodes (either density may be null).
void fmm_apply_nodes(dc_scene_s& s, const double* sigma, const double* mu, double* y,
                     const dc_eval_opts& o, hipStream_t st);
void fmm_render(dc_scene_s& s, const dc_viewport& vp, const dc_eval_opts& o, int out_dtype,
                void* out, hipStream_t st);
// dc_render without allocating: device scratch from a fixed array of
// DC_NOALLOC_SCRATCH_BYTES, every launch on st (throws DC_ERR_INVALID when
// the scene is not prepared for o's order and precision, or the render needs
// more scratch).
void fmm_render_noalloc(dc_scene_s& s, const dc_viewport& vp, const dc_eval_opts& o,
                        int out_dtype, void* out, hipStream_t st);
// Render of n viewports in one set of launches (outs[v] is [H][W][3]).
void fmm_render_batch(dc_scene_s& s, const dc_viewport* vps, int n, const dc_eval_opts& o,
                      int out_dtype, void* const* outs, hipStream_t st);
// Plan a render of n viewports (host only; throws DC_ERR_INVALID for a
// viewport outside the quadtree root).
void plan_render(const FmmState& f, const dc_viewport* vps, int n, int tile_px, int p,
                 RenderPlan& pl);
// Upward pass of the resident densities for the options' order and
// precision (a no-op when already done).
void fmm_prepare(dc_scene_s& s, const dc_eval_opts& o, hipStream_t st);
// Launch a planned render on st: scratch is device memory of
// pl.scratch_bytes and stage pinned host memory holding pl.write_tables();
// both must stay untouched until the launch has run.  Needs fmm_prepare for
// the same options first when other streams may render the scene.
void fmm_launch_render(dc_scene_s& s, const RenderPlan& pl, const dc_eval_opts& o,
                       int out_dtype, char* scratch, const void* stage, hipStream_t st);
// Run one render with device work counters; fills counts (synchronous).
void fmm_render_counts(dc_scene_s& s, const dc_viewport& vp, const dc_eval_opts& o,
                       dc_work_counts* counts, hipStream_t st);

}  // namespace dc
