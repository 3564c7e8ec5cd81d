// wmb_runtime.hip -- host runtime behind the C ABI of include/wmb.h: context,
// patch tables, launch plans (work lists), ghost-exchange plan, dt and
// diagnostics plumbing, HIP-graph capture of one step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/wmb.h"
#include "wmb_internal.h"

namespace wmb {
template <typename R> hipError_t launch_fill(void*, const PatchDev*, const WorkItem* const[3], const int[3], int, int, int, hipStream_t);
template <typename R> hipError_t launch_dt_reduce(void*, const PatchDev*, const WorkItem*, int, const DevParams&, int, unsigned long long*, hipStream_t);
hipError_t launch_dt_finalize(unsigned long long*, StepConst*, const DevParams&, hipStream_t);
hipError_t launch_set_dt(StepConst*, double, const DevParams&, hipStream_t);
hipError_t launch_set_patch(PatchDev*, int, const PatchDev&, hipStream_t);
template <typename R> hipError_t launch_ct_half(void*, const PatchDev*, const WorkItem*, int, const Coef<R>&, int, int, const StepConst*, hipStream_t);
template <typename R> hipError_t launch_update(void*, const PatchDev*, const WorkItem*, int, const DevParams&, const Coef<R>&, int, const StepConst*, unsigned long long*, unsigned long long*, int, int, unsigned int*, hipStream_t);
template <typename R> hipError_t launch_sweep(int, int, void*, const PatchDev*, const WorkItem*, int, const DevParams&, const Coef<R>&, int, const StepConst*, int, int, int, unsigned long long*, hipStream_t);
template <typename R> hipError_t launch_corr_xy(void*, const PatchDev*, const WorkItem*, int, const DevParams&, const Coef<R>&, int, const StepConst*, int, int, unsigned long long*, hipStream_t);
template <typename R> hipError_t launch_march(int, int, void*, const PatchDev*, const WorkItem*, int, const DevParams&, const Coef<R>&, int, const StepConst*, int, int, int, unsigned long long*, hipStream_t);
template <typename R> hipError_t launch_diag(const void*, const PatchDev*, const WorkItem*, int, const DevParams&, int, double*, const unsigned long long*, double, double, double*, hipStream_t);
}  // namespace wmb

using namespace wmb;

namespace {

struct DevList {
    WorkItem* d = nullptr;
    int n = 0;
};

// Sweep shapes: W > 0 is the LDS pencil form with W pencils a block; W < 0
// (y and z sweeps only) the marching form with -W pencils a block, one a
// thread.  Both forms compute every face with the same arithmetic.
struct SweepGroup {
    int P, W, zlo, tlo, thi, n;
    int Wp = 0, Wm = 0;    // autotune: the fastest pencil and marching shapes alone
    int Wx[2] = {0, 0};    // autotune, x sweeps: the second and third fastest shapes alone
    DevList wl;            // every pencil of the transverse range [tlo, n+thi]^2
    std::vector<DevList> wlg;  // the same for the patches of each step group (grouped schedule)
    DevList wl_in, wl_fr;  // Step-1 x sweep only: the pencils with both transverse
                           // coords interior, and the frame around them
    // corrector x groups, with the fused x/y corrector on: its z-plane bands
    // (all patches, and per step group) and the block's rows
    int RT = 0;
    DevList wxy;
    std::vector<DevList> wxyg;
};

// What the device signal-speed maximum (smax) holds relative to the current state.
enum SmaxState { SMAX_ZERO = 0, SMAX_CLEAN = 1, SMAX_DIRTY = 2 };

// Ghost-exchange passes (x, y, z); the update kernel writes the x-ghosts of
// the state it produces, so a fill after a step needs only FILL_YZ.
enum { FILL_X = 1, FILL_YZ = 6, FILL_ALL = 7 };

// Box of each box kernel, interior-relative [lo, n + hi]
const Box BOX_INTERIOR{0, -1};

}  // namespace

struct wmb_ctx {
    wmb_params p{};
    DevParams dp{};
    size_t esize = 8;
    bool inited = false;
    int npatch = 0;
    std::vector<wmb_patch_desc> desc;
    std::vector<PatchDev> hpatch;
    void* pool = nullptr;
    uint64_t pool_bytes = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // second stream and fork/join events of the captured step: the y/z ghost
    // exchange runs beside the interior part of the Step-1 x sweep
    hipStream_t side = nullptr, side2 = nullptr;  // borrowed from the device's spare streams
    int device = -1;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_br[6] = {};  // fork/join of the three sweep branches of a stage
    int cur = 0;
    PatchDev* d_patch = nullptr;
    DevList wl_fill[3];
    DevList wl_int, wl_diag, wl_cth, wl_upd;
    // grouped schedule (wmb_set_schedule): ngroups > 1 patch groups (whole
    // x-rows), each running its whole step on its own stream in the graph
    int ngroups = 1;
    std::vector<int> pgroup;  // patch -> step group
    std::vector<DevList> wl_cth_g, wl_upd_g;  // per step group (sized for ngroups)
    bool serial = false;  // scratch groups: the groups' steps run one after another on the main stream
    hipStream_t gstream[4] = {};  // group streams 1..3 (group 0 runs on the main stream), borrowed
    hipEvent_t ev_g[4] = {};
    int upd_zones = 256;  // zones a tile plane of Steps 8-11 (the update's block size)
    int cth_tx = 40;      // widest tile of Steps 3-4 along x (zones; 256 a tile plane)
    int upd_queue = 0;    // Steps 8-11 launch: 0 one block a tile, 1 persistent blocks on per-XCD queues
    int xy_rows = 0;      // fused x/y corrector: 0 off (separate x and y sweeps), else the most y-face rows a band
    unsigned int* d_queue = nullptr;  // the queues' counters, 16 per step group
    int nfrozen = 0;      // frozen patches
    bool plan_dirty = false;  // the active set changed since the stage work lists were planned
    bool keep_edges = false;  // Steps 8-11 also store the Step-9 edges (debugging)
    bool xg_valid = false;    // the current copy's x-ghosts (interior rows) hold the neighbours' values
    bool edges_kept = false;  // the last step stored them
    int smax_state = SMAX_ZERO;
    std::vector<SweepGroup> sweeps[3][2];
    unsigned long long* d_smax = nullptr;
    StepConst* d_sc = nullptr;
    Coef<float> cf32{};
    Coef<double> cf64{};
    unsigned long long* d_nfloor = nullptr;
    double* d_partial = nullptr;   // diagnostics records, DIAG_REC doubles per item of wl_diag
    double* d_diag_out = nullptr;  // the 12 diagnostics outputs
    double* noalloc_rec = nullptr; // this device's copy of the static records (wmb_diagnostics_noalloc)
    long long nzones = 0;          // interior zones of the batch
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    std::string err;
    std::vector<void*> owned;  // library-owned device allocations
    hipEvent_t* marks = nullptr;  // when set, an event is recorded after every kernel class
    int mark_cap = 0;             // events at marks
    int nmark = 0;
};

namespace {

template <typename R> const Coef<R>& coef(const wmb_ctx* c);
template <> const Coef<float>& coef<float>(const wmb_ctx* c) { return c->cf32; }
template <> const Coef<double>& coef<double>(const wmb_ctx* c) { return c->cf64; }

template <typename R>
void make_coef(const wmb_params& p, Coef<R>& cf) {
    cf.gam = (R)p.gamma;
    cf.gm1 = (R)(p.gamma - 1.0);
    cf.gm2 = (R)(p.gamma - 2.0);
    cf.ggm = (R)(p.gamma / (p.gamma - 1.0));
    cf.igm1 = (R)(1.0 / (p.gamma - 1.0));
    cf.beta_l = (R)p.limiter_beta;
    cf.p_floor = (R)p.p_floor;
    cf.rho_floor = (R)p.rho_floor;
    cf.tol = (R)p.degen_tol;
    cf.tol2 = (R)(p.degen_tol * p.degen_tol);
    for (int a = 0; a < 3; a++) cf.idx[a] = (R)(1.0 / p.dx[a]);
    for (int k = 0; k < 7; k++) {
        cf.eps[k] = (R)p.eps[k];
        cf.q4e[k] = p.eps[k] > 0.0 ? (R)(0.25 / p.eps[k]) : (R)0;
    }
    cf.rho_prot = (R)p.rho_protect;
    cf.p_prot = (R)p.p_protect;
}

int fail(wmb_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

// failure with a fixed message, without allocating (the message buffer is
// reserved when the context is created)
int fail_static(wmb_ctx* c, int code, const char* msg) {
    if (c) c->err.assign(msg);
    return code;
}

#define CKH(call)                                                                                           \
    do {                                                                                                    \
        hipError_t e_ = (call);                                                                             \
        if (e_ != hipSuccess)                                                                               \
            return fail(c, WMB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));                    \
    } while (0)

template <typename T>
int dev_alloc(wmb_ctx* c, T** ptr, size_t count) {
    void* p = nullptr;
    size_t bytes = sizeof(T) * (count ? count : 1);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return fail(c, WMB_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    c->owned.push_back(p);
    *ptr = static_cast<T*>(p);
    return WMB_OK;
}

// free a library-owned device allocation before the context ends
void release(wmb_ctx* c, void* p) {
    if (!p) return;
    auto it = std::find(c->owned.begin(), c->owned.end(), p);
    if (it == c->owned.end()) return;
    c->owned.erase(it);
    (void)hipFree(p);  // a list no launch uses any more: nothing to report
}

// Workgroups are dispatched to the 8 XCDs round-robin by workgroup id, and
// each XCD has its own L2.  Reorder a work list so that all blocks of a unit
// (a patch, or a group of patches the caller names) run on one XCD, in their
// original order: block id 8 j + x takes the j-th item of XCD x's queue.
// Units go to XCDs by their work in this list (items, or for column tiles
// zones x planes), largest first, each to the least loaded XCD (so that
// neither the patch numbering nor uneven patch sizes leave XCDs idle); each
// queue takes its units largest first.  Queues are padded with empty items
// (patch = -1) that exit at once.
constexpr int NXCD = 8;
std::vector<WorkItem> xcd_order(const std::vector<WorkItem>& items, const std::vector<int>* group = nullptr,
                                bool tiles = false) {
    // work and first appearance of every unit in the list
    std::vector<int> slot;  // unit -> index in order
    std::vector<long long> work;
    std::vector<std::vector<WorkItem>> per;
    for (const WorkItem& w : items) {
        const int u = group ? (*group)[w.patch] : w.patch;
        if (u >= (int)slot.size()) slot.resize(u + 1, -1);
        if (slot[u] < 0) {
            slot[u] = (int)per.size();
            per.emplace_back();
            work.push_back(0);
        }
        const long long wt = tiles ? (long long)(w.b & 0xffff) * (w.b >> 16) * ((w.c >> 16) - (w.c & 0xffff)) : 1;
        work[slot[u]] += wt;
        per[slot[u]].push_back(w);
    }
    std::vector<int> byload(per.size());
    for (size_t i = 0; i < byload.size(); i++) byload[i] = (int)i;
    std::stable_sort(byload.begin(), byload.end(), [&](int a, int b) { return work[a] > work[b]; });
    long long load[NXCD] = {0};
    std::vector<std::vector<WorkItem>> q(NXCD);
    for (int i : byload) {
        int best = 0;
        for (int x = 1; x < NXCD; x++)
            if (load[x] < load[best]) best = x;
        load[best] += work[i];
        for (const WorkItem& w : per[i]) q[best].push_back(w);
    }
    size_t len = 0;
    for (auto& v : q) len = v.size() > len ? v.size() : len;
    std::vector<WorkItem> out;
    out.reserve(len * NXCD);
    for (size_t j = 0; j < len; j++)
        for (int x = 0; x < NXCD; x++) out.push_back(j < q[x].size() ? q[x][j] : WorkItem{-1, 0, 0, 0});
    return out;
}

template <typename T>
int upload(wmb_ctx* c, T** ptr, const std::vector<T>& h) {
    int rc = dev_alloc(c, ptr, h.size());
    if (rc) return rc;
    if (!h.empty()) CKH(hipMemcpy(*ptr, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
    return WMB_OK;
}

int check_params(const wmb_params* p) {
    if (!p) return WMB_EINVAL;
    if (!(p->gamma > 1.0) || !(p->cfl > 0.0 && p->cfl <= 1.0)) return WMB_EINVAL;
    if (p->ghost < 4 || p->ghost > 16) return WMB_EINVAL;
    for (int a = 0; a < 3; a++)
        if (!(p->dx[a] > 0.0)) return WMB_EINVAL;
    for (int k = 0; k < 7; k++)
        if (!(p->eps[k] >= 0.0 && p->eps[k] < 0.5)) return WMB_EINVAL;
    if (!(p->limiter_beta >= 1.0 && p->limiter_beta <= 2.0)) return WMB_EINVAL;
    if (!(p->rho_floor > 0.0) || !(p->p_floor > 0.0)) return WMB_EINVAL;
    if (!(p->degen_tol >= 0.0 && p->degen_tol < 1e-2)) return WMB_EINVAL;
    if (p->precision != WMB_FP64 && p->precision != WMB_FP32) return WMB_EINVAL;
    if (!(p->rho_protect >= 0.0) || !(p->p_protect >= 0.0)) return WMB_EINVAL;
    if (p->dt_lag != 0 && p->dt_lag != 1) return WMB_EINVAL;
    if (p->scratch_groups < 0 || p->scratch_groups > 64) return WMB_EINVAL;
    return WMB_OK;
}

size_t esize_of(const wmb_params* p) { return p->precision == WMB_FP32 ? 4 : 8; }

long long vol_of(const wmb_patch_desc& d, int g) {
    return (long long)(d.n[0] + 2 * g) * (d.n[1] + 2 * g) * (d.n[2] + 2 * g);
}

// a patch's state region and its space for the step's intermediates, in
// bytes, rounded to 256 B
uint64_t align256(uint64_t b) { return (b + 255) & ~uint64_t(255); }
uint64_t state_bytes(const wmb_patch_desc& d, int g, size_t es) {
    return align256((uint64_t)F_STATE * (uint64_t)vol_of(d, g) * es);
}
uint64_t scratch_bytes(const wmb_patch_desc& d, int g, size_t es) {
    return align256((uint64_t)F_SCRATCH * (uint64_t)vol_of(d, g) * es);
}

// x-rows: patches linked by their x face neighbours in the init table (a
// periodic ring or a chain between domain boundaries), named by their
// lowest member
std::vector<int> rows_of(int np, const wmb_patch_desc* d) {
    std::vector<int> row(np, -1), seen(np, -1);
    const int fx[2] = {12, 14};
    for (int p = 0; p < np; p++) {
        if (row[p] >= 0) continue;
        std::vector<int> members{p};
        seen[p] = p;
        for (int dir = 0; dir < 2; dir++)  // walk -x, then +x
            for (int q = d[p].nbr[fx[dir]]; q >= 0 && q < np && seen[q] != p; q = d[q].nbr[fx[dir]]) {
                seen[q] = p;
                members.push_back(q);
            }
        const int id = *std::min_element(members.begin(), members.end());
        for (int m : members) row[m] = id;
    }
    return row;
}

// whole x-rows dealt to `groups` groups in turn, in the order of their first patch
std::vector<int> deal_rows(int np, const wmb_patch_desc* d, int groups) {
    const std::vector<int> rows = rows_of(np, d);
    std::vector<int> ord(np, -1), grp(np, 0);
    int next = 0;
    for (int p = 0; p < np; p++) {
        if (ord[rows[p]] < 0) ord[rows[p]] = next++;
        grp[p] = groups > 1 ? ord[rows[p]] % groups : 0;
    }
    return grp;
}

// The pool.  Without scratch groups every patch has one region: its state,
// then its intermediates (a patch's arrays stay close together in memory:
// with all intermediates after all states, Steps 3-4 and 8-11 measured 1-2%
// slower at 256^3 FP32).  With scratch groups the patches' state regions come one
// after another, then one set of intermediate slots per group, all groups at
// the same addresses (their steps run one after another), as large as the
// largest group's.  Byte offsets.
struct PoolLayout {
    std::vector<uint64_t> base, sbase;
    uint64_t total = 0;
};
PoolLayout plan_pool(int np, const wmb_patch_desc* d, int g, size_t es, int groups) {
    PoolLayout L;
    L.base.resize(np);
    L.sbase.resize(np);
    uint64_t off = 0;
    if (groups <= 1) {
        for (int p = 0; p < np; p++) {
            L.base[p] = off;
            off += state_bytes(d[p], g, es);
            L.sbase[p] = off;
            off += scratch_bytes(d[p], g, es);
        }
        L.total = off;
        return L;
    }
    for (int p = 0; p < np; p++) {
        L.base[p] = off;
        off += state_bytes(d[p], g, es);
    }
    const std::vector<int> grp = deal_rows(np, d, groups);
    std::vector<uint64_t> fill(groups, 0);
    uint64_t top = 0;
    for (int p = 0; p < np; p++) {
        L.sbase[p] = off + fill[grp[p]];
        fill[grp[p]] += scratch_bytes(d[p], g, es);
        top = std::max(top, fill[grp[p]]);
    }
    L.total = off + top;
    return L;
}

// Largest interior edge the kernels take, per precision.  Every axis is a
// transverse axis of some sweep, and a sweep work item packs its pencil
// rectangle's first transverse coordinates as 10-bit fields biased by 512,
// where a frame rectangle starts at the edge n itself: n <= 511.  A Step-1
// sweep block holds whole pencils of n + 8 zones with 16 words of LDS a zone
// (at most 1024 threads and 64 KiB): n <= 1016 in FP32, n <= 504 in FP64.
int max_edge(size_t es) { return es == 4 ? 511 : 504; }

int check_table(int32_t np, const wmb_patch_desc* d, int g, size_t es, std::string& why) {
    for (int i = 0; i < np; i++) {
        for (int a = 0; a < 3; a++)
            if (d[i].n[a] < g || d[i].n[a] > max_edge(es)) {
                why = "patch " + std::to_string(i) + ": interior edge below the ghost width or above " +
                      std::to_string(max_edge(es));
                return WMB_EINVAL;
            }
        // kernels address a patch's regions with 32-bit byte offsets
        if (scratch_bytes(d[i], g, es) > 0xFFFFFFFFull) {
            why = "patch " + std::to_string(i) + ": region above 4 GiB (32-bit offsets)";
            return WMB_EINVAL;
        }
        if (d[i].nbr[13] != i) {
            why = "patch " + std::to_string(i) + ": nbr[13] must be the patch itself";
            return WMB_EINVAL;
        }
        for (int t = 0; t < 27; t++)
            if (d[i].nbr[t] < -1 || d[i].nbr[t] >= np) {
                why = "patch " + std::to_string(i) + ": neighbour id out of range";
                return WMB_EINVAL;
            }
    }
    // every id is in range from here on, so the chains below index d safely
    for (int i = 0; i < np; i++) {
        for (int t = 0; t < 27; t++) {
            int q = d[i].nbr[t];
            int off[3] = {t % 3 - 1, (t / 3) % 3 - 1, t / 9 - 1};
            // edge and corner neighbours are reached through face neighbours
            // (z, then y, then x): the ghost exchange copies along that chain;
            // a step that leaves the domain (-1, a domain boundary) makes the
            // entry -1
            int r = i;
            if (off[2] && r >= 0) r = d[r].nbr[9 * (off[2] + 1) + 4];
            if (off[1] && r >= 0) r = d[r].nbr[9 + 3 * (off[1] + 1) + 1];
            if (off[0] && r >= 0) r = d[r].nbr[12 + off[0] + 1];
            if (r != q) {
                why = "patch " + std::to_string(i) + ": edge/corner neighbour inconsistent with the face neighbours";
                return WMB_EINVAL;
            }
            if (q < 0) continue;
            for (int a = 0; a < 3; a++)
                if (off[a] == 0 && d[q].n[a] != d[i].n[a]) {
                    why = "patch " + std::to_string(i) + ": neighbour " + std::to_string(q) + " extent mismatch";
                    return WMB_EINVAL;
                }
            // the neighbour in the opposite direction of my neighbour is me
            int back = 9 * (1 - off[2]) + 3 * (1 - off[1]) + (1 - off[0]);
            if (d[q].nbr[back] != i) {
                why = "patch " + std::to_string(i) + ": neighbour table not symmetric";
                return WMB_EINVAL;
            }
        }
    }
    return WMB_OK;
}

// profiling marks only (wmb_profile_step checks the events it reads)
void mark(wmb_ctx* c) {
    if (c->marks && c->nmark < c->mark_cap) (void)hipEventRecord(c->marks[c->nmark], c->stream);
    if (c->marks) c->nmark++;
}

template <typename R>
hipError_t launch_group(wmb_ctx* c, int d, int stage, const SweepGroup& G, const DevList& L, int cur,
                        unsigned long long* nprot, hipStream_t st) {
    if (G.W < 0)
        return launch_march<R>(d, stage, c->pool, c->d_patch, L.d, L.n, c->dp, coef<R>(c), cur, c->d_sc, G.P, -G.W,
                               G.zlo, nprot, st);
    return launch_sweep<R>(d, stage, c->pool, c->d_patch, L.d, L.n, c->dp, coef<R>(c), cur, c->d_sc, G.P, G.W, G.zlo,
                           nprot, st);
}

// with the fused x/y corrector on, the z predictor records it stores are
// what the z corrector reads (stage 3), so the z sweep follows it
bool zrec(const wmb_ctx* c) { return c->xy_rows > 0; }

// the z corrector sweeps of one group's list: from the stored records after
// the fused x/y corrector, else from q^n and the Step-1 fluxes
template <typename R>
hipError_t launch_corr_z(wmb_ctx* c, int g, int cur, unsigned long long* nprot, hipStream_t st) {
    for (auto& G : c->sweeps[2][1]) {
        hipError_t r = launch_group<R>(c, 2, zrec(c) ? 3 : 2, G, g < 0 ? G.wl : G.wlg[g], cur, nprot, st);
        if (r != hipSuccess) return r;
    }
    return hipSuccess;
}

// the corrector's x sweeps of one group's list (wl: all patches; g >= 0: step
// group g), as the fused x/y kernel when xy_rows > 0
template <typename R>
hipError_t launch_corr_x(wmb_ctx* c, int g, int cur, unsigned long long* nprot, hipStream_t st) {
    for (auto& G : c->sweeps[0][1]) {
        hipError_t r;
        if (c->xy_rows > 0) {
            const DevList& L = g < 0 ? G.wxy : G.wxyg[g];
            r = launch_corr_xy<R>(c->pool, c->d_patch, L.d, L.n, c->dp, coef<R>(c), cur, c->d_sc, G.P, G.RT, nprot,
                                  st);
        } else {
            r = launch_group<R>(c, 0, 2, G, g < 0 ? G.wl : G.wlg[g], cur, nprot, st);
        }
        if (r != hipSuccess) return r;
    }
    return hipSuccess;
}

// whether a sweep shape is valid for axis d and pencils of P zones (marching
// shapes -W with W in [1, 256], or W + 512 in FP32 for the corrector with
// the next zone's loads issued one zone ahead)
bool shape_ok(int d, int P, size_t es, int W, int stage) {
    if (W < 0) {
        const int w = -W;
        return d != 0 && ((w >= 1 && w <= 256) || (es == 4 && stage == 2 && w >= 513 && w <= 768));
    }
    return W >= 1 && (size_t)P * W <= 1024 && es * 16 * (size_t)P * W <= 64 * 1024;
}

template <typename R>
int run_fill(wmb_ctx* c, int mask) {
    const WorkItem* wl[3] = {c->wl_fill[0].d, c->wl_fill[1].d, c->wl_fill[2].d};
    const int nw[3] = {c->wl_fill[0].n, c->wl_fill[1].n, c->wl_fill[2].n};
    hipError_t e = launch_fill<R>(c->pool, c->d_patch, wl, nw, c->p.ghost, c->cur, mask, c->stream);
    if (e != hipSuccess) return fail(c, WMB_EHIP, std::string("fill_ghosts: ") + hipGetErrorString(e));
    if (mask & FILL_X) c->xg_valid = true;
    mark(c);
    return WMB_OK;
}

// make smax the signal-speed maximum of the current state (explicit reduction)
template <typename R>
int run_reduce(wmb_ctx* c) {
    hipError_t e = launch_dt_reduce<R>(c->pool, c->d_patch, c->wl_int.d, c->wl_int.n, c->dp, c->cur, c->d_smax, c->stream);
    if (e != hipSuccess) return fail(c, WMB_EHIP, std::string("dt_reduce: ") + hipGetErrorString(e));
    c->smax_state = SMAX_CLEAN;
    return WMB_OK;
}

// dt = cfl / smax (smax then reset to zero)
int run_finalize(wmb_ctx* c) {
    hipError_t e = launch_dt_finalize(c->d_smax, c->d_sc, c->dp, c->stream);
    if (e != hipSuccess) return fail(c, WMB_EHIP, std::string("dt_finalize: ") + hipGetErrorString(e));
    c->smax_state = SMAX_ZERO;
    mark(c);
    return WMB_OK;
}

// one sweep group's launch in its form
template <typename R>
hipError_t launch_group(wmb_ctx* c, int d, int stage, const SweepGroup& G, const DevList& L, int cur,
                        unsigned long long* nprot, hipStream_t st);

// One step.  split (the captured graph): the y/z ghost exchange was forked
// onto the side stream (ev_join marks its end).  The three sweeps of a stage
// are independent (each writes its own flux array), so they run as three
// branches: x on the main stream, y on the side stream, z on the second side
// stream, joined before Steps 3-4 and before Steps 8-11 (with the fused
// corrector, Steps 5-7 are its launch and then the z sweep from its records,
// both on the main stream).  The Step-1 x sweep
// first covers the pencils whose transverse coords are interior, which read
// only the x-ghosts the previous update wrote, then waits for the exchange
// and covers the frame.
template <typename R>
int run_step(wmb_ctx* c, bool split = false) {
    hipError_t e;
    const int cur = c->cur;
#define STEPCK(what)                                                                        \
    if (e != hipSuccess) return fail(c, WMB_EHIP, std::string(what) + ": " + hipGetErrorString(e))
    auto sweeps = [&](int d, int stage, const DevList SweepGroup::*wl, hipStream_t st) -> hipError_t {
        for (auto& G : c->sweeps[d][stage - 1]) {
            const DevList& L = G.*wl;
            hipError_t r = launch_group<R>(c, d, stage, G, L, cur, c->d_nfloor + 1, st);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    };
    if (split) {
        // Step 1: y after the exchange on its stream, z waits for it on the
        // second; both also wait for this step's dt (finalized on the main
        // stream before this call)
        CKH(hipEventRecord(c->ev_br[5], c->stream));
        CKH(hipStreamWaitEvent(c->side, c->ev_br[5], 0));
        CKH(hipStreamWaitEvent(c->side2, c->ev_br[5], 0));
        CKH(hipStreamWaitEvent(c->side2, c->ev_join, 0));
        e = sweeps(1, 1, &SweepGroup::wl, c->side);
        STEPCK("sweep1");
        e = sweeps(2, 1, &SweepGroup::wl, c->side2);
        STEPCK("sweep1");
        CKH(hipEventRecord(c->ev_br[0], c->side));
        CKH(hipEventRecord(c->ev_br[1], c->side2));
        e = sweeps(0, 1, &SweepGroup::wl_in, c->stream);
        STEPCK("sweep1");
        CKH(hipStreamWaitEvent(c->stream, c->ev_join, 0));
        e = sweeps(0, 1, &SweepGroup::wl_fr, c->stream);
        STEPCK("sweep1");
        CKH(hipStreamWaitEvent(c->stream, c->ev_br[0], 0));
        CKH(hipStreamWaitEvent(c->stream, c->ev_br[1], 0));
    } else {
        for (int d = 0; d < 3; d++) {
            e = sweeps(d, 1, &SweepGroup::wl, c->stream);
            STEPCK("sweep1");
            mark(c);
        }
    }
    e = launch_ct_half<R>(c->pool, c->d_patch, c->wl_cth.d, c->wl_cth.n, coef<R>(c), c->p.ghost, cur, c->d_sc, c->stream);
    STEPCK("ct_half");
    mark(c);
    if (split) {
        CKH(hipEventRecord(c->ev_br[2], c->stream));
        CKH(hipStreamWaitEvent(c->side, c->ev_br[2], 0));
        CKH(hipStreamWaitEvent(c->side2, c->ev_br[2], 0));
        // with the fused x/y corrector the y branch is empty; when it stores
        // the z records, the z corrector follows it on the main stream
        if (!c->xy_rows) {
            e = sweeps(1, 2, &SweepGroup::wl, c->side);
            STEPCK("sweep2");
        }
        if (!zrec(c)) {
            e = launch_corr_z<R>(c, -1, cur, c->d_nfloor + 1, c->side2);
            STEPCK("sweep2");
        }
        CKH(hipEventRecord(c->ev_br[3], c->side));
        CKH(hipEventRecord(c->ev_br[4], c->side2));
        e = launch_corr_x<R>(c, -1, cur, c->d_nfloor + 1, c->stream);
        STEPCK("sweep2");
        if (zrec(c)) {
            e = launch_corr_z<R>(c, -1, cur, c->d_nfloor + 1, c->stream);
            STEPCK("sweep2");
        }
        CKH(hipStreamWaitEvent(c->stream, c->ev_br[3], 0));
        CKH(hipStreamWaitEvent(c->stream, c->ev_br[4], 0));
    } else {
        for (int d = 0; d < 3; d++) {
            if (d == 0) e = launch_corr_x<R>(c, -1, cur, c->d_nfloor + 1, c->stream);
            else if (d == 2) e = launch_corr_z<R>(c, -1, cur, c->d_nfloor + 1, c->stream);
            else if (!c->xy_rows) e = sweeps(d, 2, &SweepGroup::wl, c->stream);
            STEPCK("sweep2");
            mark(c);
        }
    }
    e = launch_update<R>(c->pool, c->d_patch, c->wl_upd.d, c->wl_upd.n, c->dp, coef<R>(c), cur, c->d_sc, c->d_nfloor,
                         c->d_smax, c->keep_edges ? 1 : 0, c->upd_zones, c->upd_queue ? c->d_queue : nullptr,
                         c->stream);
    STEPCK("update");
    mark(c);
    c->edges_kept = c->keep_edges;
    c->xg_valid = true;  // the update wrote the x-ghosts of the new copy
#undef STEPCK
    c->cur ^= 1;
    // the final update folds the new state's signal speeds into smax
    c->smax_state = (c->smax_state == SMAX_ZERO) ? SMAX_CLEAN : SMAX_DIRTY;
    return WMB_OK;
}

// The grouped schedule of the step: the patch groups (whole x-rows) run
// their whole step (Step-1 sweeps, Steps 3-4, Steps 5-7, Steps 8-11) each on
// its own stream, forked after dt and joined before the next exchange, so
// that one group's memory-bound stages overlap another's sweeps.  Within a
// step a patch's kernels touch only its own region, apart from the update's
// x-ghost pushes, which write the neighbours' other state copy (read only
// after the join), so the groups share no data inside the step.  With
// scratch groups (serial) the groups share the space for the intermediates,
// so they run one after another on the main stream.
template <typename R>
int run_step_grouped(wmb_ctx* c) {
    const int cur = c->cur;
    const bool par = !c->serial;
    if (par) {
        CKH(hipEventRecord(c->ev_fork, c->stream));
        for (int g = 1; g < c->ngroups; g++) CKH(hipStreamWaitEvent(c->gstream[g], c->ev_fork, 0));
    }
    for (int g = 0; g < c->ngroups; g++) {
        hipStream_t st = (g == 0 || !par) ? c->stream : c->gstream[g];
        hipError_t e = hipSuccess;
        for (int stage = 1; stage <= 2 && e == hipSuccess; stage++) {
            for (int d = 0; d < 3 && e == hipSuccess; d++) {
                if (stage == 2 && d == 0) {
                    e = launch_corr_x<R>(c, g, cur, c->d_nfloor + 1, st);
                } else if (stage == 2 && d == 2) {
                    e = launch_corr_z<R>(c, g, cur, c->d_nfloor + 1, st);
                } else if (!(stage == 2 && d == 1 && c->xy_rows)) {
                    for (auto& SG : c->sweeps[d][stage - 1])
                        if (e == hipSuccess) e = launch_group<R>(c, d, stage, SG, SG.wlg[g], cur, c->d_nfloor + 1, st);
                }
                if (!par) mark(c);
            }
            if (stage == 1 && e == hipSuccess) {
                e = launch_ct_half<R>(c->pool, c->d_patch, c->wl_cth_g[g].d, c->wl_cth_g[g].n, coef<R>(c), c->p.ghost,
                                      cur, c->d_sc, st);
                if (!par) mark(c);
            }
        }
        const DevList& wu = c->wl_upd_g[g];
        if (e == hipSuccess)
            e = launch_update<R>(c->pool, c->d_patch, wu.d, wu.n, c->dp, coef<R>(c), cur, c->d_sc, c->d_nfloor, c->d_smax,
                                 c->keep_edges ? 1 : 0, c->upd_zones,
                                 c->upd_queue ? c->d_queue + 16 * (par ? g : 0) : nullptr, st);
        if (!par) mark(c);
        if (e != hipSuccess) return fail(c, WMB_EHIP, std::string("grouped step: ") + hipGetErrorString(e));
        if (g > 0 && par) CKH(hipEventRecord(c->ev_g[g], st));
    }
    if (par)
        for (int g = 1; g < c->ngroups; g++) CKH(hipStreamWaitEvent(c->stream, c->ev_g[g], 0));
    c->edges_kept = c->keep_edges;
    c->xg_valid = true;
    c->cur ^= 1;
    c->smax_state = (c->smax_state == SMAX_ZERO) ? SMAX_CLEAN : SMAX_DIRTY;
    return WMB_OK;
}

int dispatch_fill(wmb_ctx* c, int mask = FILL_ALL) {
    return c->esize == 4 ? run_fill<float>(c, mask) : run_fill<double>(c, mask);
}
int ensure_smax(wmb_ctx* c) {
    if (c->smax_state == SMAX_CLEAN) return WMB_OK;
    return c->esize == 4 ? run_reduce<float>(c) : run_reduce<double>(c);
}
int dispatch_dt(wmb_ctx* c) {
    int rc = ensure_smax(c);
    return rc ? rc : run_finalize(c);
}
int dispatch_step(wmb_ctx* c, bool split = false) {
    if ((split || c->serial) && c->ngroups > 1)
        return c->esize == 4 ? run_step_grouped<float>(c) : run_step_grouped<double>(c);
    return c->esize == 4 ? run_step<float>(c, split) : run_step<double>(c, split);
}
// the y/z ghost exchange on the side stream, forked from and joined (by the
// split step, through ev_join) back into the main stream
int fork_fill_yz(wmb_ctx* c) {
    const WorkItem* wl[3] = {c->wl_fill[0].d, c->wl_fill[1].d, c->wl_fill[2].d};
    const int nw[3] = {c->wl_fill[0].n, c->wl_fill[1].n, c->wl_fill[2].n};
    CKH(hipEventRecord(c->ev_fork, c->stream));
    CKH(hipStreamWaitEvent(c->side, c->ev_fork, 0));
    hipError_t e = c->esize == 4 ? launch_fill<float>(c->pool, c->d_patch, wl, nw, c->p.ghost, c->cur, FILL_YZ, c->side)
                                 : launch_fill<double>(c->pool, c->d_patch, wl, nw, c->p.ghost, c->cur, FILL_YZ, c->side);
    if (e != hipSuccess) return fail(c, WMB_EHIP, std::string("fill_ghosts: ") + hipGetErrorString(e));
    CKH(hipEventRecord(c->ev_join, c->side));
    return WMB_OK;
}

int build_box_list(wmb_ctx* c, Box bx, DevList& out, bool xcd = true) {
    std::vector<WorkItem> items;
    for (int p = 0; p < c->npatch; p++) {
        long long e = 1;
        for (int a = 0; a < 3; a++) e *= (long long)(c->desc[p].n[a] + bx.hi - bx.lo + 1);
        int nb = (int)((e + 255) / 256);
        for (int b = 0; b < nb; b++) items.push_back(WorkItem{p, b, 0, 0});
    }
    if (xcd) items = xcd_order(items);
    out.n = (int)items.size();
    return upload(c, &out.d, items);
}

// Diagnostics work items: runs of at most DIAG_CHUNK interior zones of one
// patch (linear index, x fastest): a = first zone, b = count.  Patch order,
// so that the reduction order is fixed.
constexpr int DIAG_CHUNK = 32768;
int build_diag_list(wmb_ctx* c) {
    std::vector<WorkItem> items;
    for (int p = 0; p < c->npatch; p++) {
        const int nz = c->desc[p].n[0] * c->desc[p].n[1] * c->desc[p].n[2];
        for (int z0 = 0; z0 < nz; z0 += DIAG_CHUNK) items.push_back(WorkItem{p, z0, std::min(DIAG_CHUNK, nz - z0), 0});
    }
    c->wl_diag.n = (int)items.size();
    return upload(c, &c->wl_diag.d, items);
}

// Column tiles of the marching kernels over the in-plane box [lo, n+hi]^2
// (x, y) and the planes [zlo, n+zhi]: each patch's box is cut into near-equal
// parts of at most txmax zones along x (whole rows where they fit, so tile
// rows cut no cache lines), then along y into parts with at most maxz zones
// per tile plane and 32 per edge.  Item fields (origins biased by 16, they
// may be negative): a = i0 | j0 << 16, b = tx | ty << 16, c = k0 | k1 << 16
// with k1 exclusive.
constexpr int TILE_BIAS = 16;
// x-rows: patches linked by their x face neighbours (a periodic ring or a
// chain between domain boundaries), numbered by their smallest patch id;
// the unit of xcd_order for the update and the ghost exchange
std::vector<int> x_rows(const wmb_ctx* c) { return rows_of(c->npatch, c->desc.data()); }

// The stage work lists (sweeps, Steps 3-4, Steps 8-11) cover the present,
// active patches; frozen and absent ones are left out when the lists are
// planned again (replan), so their blocks are not launched at all.
bool in_plan(const wmb_ctx* c, int p) { return c->hpatch[p].present && c->hpatch[p].active; }

std::vector<WorkItem> tile_items(const wmb_ctx* c, int lo, int hi, int zlo, int zhi, int txmax_allowed, int maxz,
                                 const std::vector<int>* group, int sgroup = -1, int ermax = 0, int edmax = 0) {
    std::vector<WorkItem> items;
    for (int p = 0; p < c->npatch; p++) {
        if (!in_plan(c, p) || (sgroup >= 0 && c->pgroup[p] != sgroup)) continue;
        const int* n = c->desc[p].n;
        const int ex = n[0] + hi - lo + 1, ey = n[1] + hi - lo + 1;
        const int mx = (ex + txmax_allowed - 1) / txmax_allowed;
        const int txmax = (ex + mx - 1) / mx;
        int tymax = maxz / txmax;
        if (tymax > 32) tymax = 32;
        // LDS planes of the Steps 8-11 kernel: E^r with its ring, the edges
        if (ermax > 0) tymax = std::min(tymax, ermax / (txmax + 2) - 2);
        if (edmax > 0) tymax = std::min(tymax, edmax / (txmax + 1) - 1);
        const int my = (ey + tymax - 1) / tymax;
        const int k0 = zlo + TILE_BIAS, k1 = n[2] + zhi + 1 + TILE_BIAS;
        for (int by = 0; by < my; by++) {
            const int j0 = lo + (int)((long long)ey * by / my), j1 = lo + (int)((long long)ey * (by + 1) / my);
            for (int bx = 0; bx < mx; bx++) {
                const int i0 = lo + (int)((long long)ex * bx / mx), i1 = lo + (int)((long long)ex * (bx + 1) / mx);
                items.push_back(WorkItem{p, (i0 + TILE_BIAS) | ((j0 + TILE_BIAS) << 16), (i1 - i0) | ((j1 - j0) << 16),
                                         k0 | (k1 << 16)});
            }
        }
    }
    return xcd_order(items, group, true);
}

int build_tile_list(wmb_ctx* c, int lo, int hi, int zlo, int zhi, int txmax_allowed, int maxz,
                    const std::vector<int>* group, DevList& out, int sgroup = -1, int ermax = 0, int edmax = 0) {
    std::vector<WorkItem> items = tile_items(c, lo, hi, zlo, zhi, txmax_allowed, maxz, group, sgroup, ermax, edmax);
    out.n = (int)items.size();
    return upload(c, &out.d, items);
}

// The Steps 8-11 tiles for tile planes of Z zones: whole rows of up to 48
// zones in the 512-zone FP32 blocks (a 48^3 patch's rows stay whole: 48 x 10
// tiles instead of 24 x 16), up to 32 otherwise, with ty capped so that the
// E^r and edge planes fit the kernel's LDS.
int upd_txmax(int Z) { return Z > 256 ? 48 : 32; }
std::vector<WorkItem> upd_items(const wmb_ctx* c, int Z, const std::vector<int>* rows, int sgroup = -1) {
    const int es = (int)c->esize;
    return tile_items(c, 0, -1, 0, -1, upd_txmax(Z), Z, rows, sgroup, upd_er_plane(es), upd_ed_plane(es));
}
int build_upd_list(wmb_ctx* c, int Z, const std::vector<int>* rows, DevList& out, int sgroup = -1) {
    std::vector<WorkItem> items = upd_items(c, Z, rows, sgroup);
    out.n = (int)items.size();
    return upload(c, &out.d, items);
}

// Zones a tile plane of Steps 8-11 (the update's block size): the largest
// that upd_tile_zones_max allows, unless the patches' tiles would leave more
// of its threads idle than 256-zone tiles do (patches whose x-y planes hold
// fewer zones than a block)
int choose_upd_zones(const wmb_ctx* c) {
    const int zmax = upd_tile_zones_max((int)c->esize);
    if (zmax <= 256) return 256;
    const int Z[2] = {256, zmax};
    double fill[2];
    for (int v = 0; v < 2; v++) {
        long long zones = 0, slots = 0;
        const int es = (int)c->esize, txa = upd_txmax(Z[v]);
        for (int p = 0; p < c->npatch; p++) {
            // the column-tile cut of upd_items for the interior x-y plane
            const int ex = c->desc[p].n[0], ey = c->desc[p].n[1];
            const int mx = (ex + txa - 1) / txa, txmax = (ex + mx - 1) / mx;
            const int tymax = std::min({32, Z[v] / txmax, upd_er_plane(es) / (txmax + 2) - 2,
                                        upd_ed_plane(es) / (txmax + 1) - 1});
            const int my = (ey + tymax - 1) / tymax;
            zones += (long long)ex * ey;
            slots += (long long)mx * my * Z[v];
        }
        fill[v] = (double)zones / (double)slots;
    }
    return fill[1] >= fill[0] ? zmax : 256;
}

// The tile lists of Steps 3-4 and 8-11 for the current cth_tx and
// upd_zones: Steps 3-4 tiles up to cth_tx zones wide and 256 a plane
// ((tx+1)(ty+1) <= 297 edges for any tx <= 40); Steps 8-11 tiles of
// upd_zones a plane as upd_items cuts them.  The update
// and the ghost exchange place whole x-rows of patches on an XCD, so that
// the update's x-ghost pushes go to a patch on the same XCD: 256^3 FP32
// update 1.14 against 1.24 ms, the uneven batch 1.80 against 2.04 ms, at the
// same measured HBM traffic (orders that put x-neighbours on other XCDs
// measured 1.24 ms at 256^3).  The sweeps keep one patch a unit, which
// measured faster for them.  With a grouped schedule, the lists of every
// group as well.
int build_ct_update_lists(wmb_ctx* c) {
    for (DevList* L : {&c->wl_cth, &c->wl_upd}) {
        release(c, L->d);
        *L = DevList{};
    }
    const std::vector<int> rows = x_rows(c);
    int rc = build_tile_list(c, -2, 2, -2, 2, c->cth_tx, 256, nullptr, c->wl_cth);
    if (!rc) rc = build_upd_list(c, c->upd_zones, &rows, c->wl_upd);
    if (c->ngroups > 1 && c->wl_cth_g.size() < (size_t)c->ngroups) {
        c->wl_cth_g.resize(c->ngroups);
        c->wl_upd_g.resize(c->ngroups);
    }
    for (int g = 0; g < c->ngroups && c->ngroups > 1 && !rc; g++) {
        for (DevList* L : {&c->wl_cth_g[g], &c->wl_upd_g[g]}) {
            release(c, L->d);
            *L = DevList{};
        }
        rc = build_tile_list(c, -2, 2, -2, 2, c->cth_tx, 256, nullptr, c->wl_cth_g[g], g);
        if (!rc) rc = build_upd_list(c, c->upd_zones, &rows, c->wl_upd_g[g], g);
    }
    return rc;
}

int build_fill_lists(wmb_ctx* c) {
    const int g = c->p.ghost;
    const std::vector<int> rows = x_rows(c);
    for (int ax = 0; ax < 3; ax++) {
        std::vector<WorkItem> items;
        for (int p = 0; p < c->npatch; p++) {
            const int* n = c->desc[p].n;
            // rows reach the owned boundary face along a later axis that ends
            // at a domain boundary on the right; the kernel takes its extents
            // from the patch table, so the list covers the longer rows always
            // (removing or adding a neighbour then needs no new list)
            const int wy = 1, wz = 1;
            long long e;
            if (ax == 0) e = 2LL * g * (n[1] + wy) * (n[2] + wz);
            else if (ax == 1) e = 2LL * g * (n[0] + 2 * g) * (n[2] + wz);
            else e = 2LL * g * (n[0] + 2 * g) * (n[1] + 2 * g);
            int nb = (int)((e + 255) / 256);
            for (int b = 0; b < nb; b++) items.push_back(WorkItem{p, b, 0, 0});
        }
        items = xcd_order(items, &rows);
        c->wl_fill[ax].n = (int)items.size();
        int rc = upload(c, &c->wl_fill[ax].d, items);
        if (rc) return rc;
    }
    return WMB_OK;
}

int choose_W(int d, int P, size_t es) {
    // y and z in FP32: the marching form (coalesced, no barrier; about 120
    // VGPRs, 4 waves a SIMD); in FP64 it needs 256 VGPRs and the pencil form
    // is kept
    if (d != 0 && es == 4) return -64;
    if (d == 0) {
        // about 256 threads a block, packed into whole 64-lane waves: the
        // pencil count whose P * W wastes the fewest lanes, nearest to 256
        int best = 256 / P < 1 ? 1 : 256 / P;
        double bs = -1.0;
        for (int W = 1; (size_t)P * W <= 1024 && es * 16 * (size_t)P * W <= 64 * 1024; W++) {
            const int t = P * W;
            if (t < 128 && (size_t)P * (W + 1) <= 1024) continue;
            const double fill = (double)t / (double)((t + 63) / 64 * 64);
            const double score = fill - 0.02 * (t > 256 ? t - 256 : 256 - t) / 64.0;
            if (score > bs) {
                bs = score;
                best = W;
            }
        }
        return best;
    }
    int W = 16;
    while (W > 1 && ((size_t)P * W > 1024 || es * 16 * (size_t)P * W > 64 * 1024)) W /= 2;
    return W;
}

// Which pencils of the transverse range [tlo, n+thi]^2 a list covers: all, the
// interior rectangle [0, n)^2, or the frame between the two.
enum SweepPart { PART_ALL, PART_INTERIOR, PART_FRAME };

// pencils of every patch whose edge along d is n, W consecutive pencils of one
// rectangle a block
// *bad is set when a pencil rectangle does not fit the packed fields
std::vector<WorkItem> sweep_items(const wmb_ctx* c, int d, int n, int tlo, int thi, int W, SweepPart part = PART_ALL,
                                  int group = -1, bool* bad = nullptr) {
    const int FA = (d == 0) ? 1 : 0;
    const int SA = (d == 0) ? 2 : (d == 1 ? 2 : 1);
    struct Rect {
        int flo, fcnt, slo, scnt;
    };
    std::vector<WorkItem> items;
    for (int p = 0; p < c->npatch; p++) {
        if (c->desc[p].n[d] != n || !in_plan(c, p)) continue;
        if (group >= 0 && c->pgroup[p] != group) continue;
        const int nf = c->desc[p].n[FA], ns = c->desc[p].n[SA];
        const int tf = nf + thi - tlo + 1;
        std::vector<Rect> rects;
        if (part == PART_ALL) rects.push_back({tlo, tf, tlo, ns + thi - tlo + 1});
        if (part == PART_INTERIOR) rects.push_back({0, nf, 0, ns});
        if (part == PART_FRAME) {
            rects.push_back({tlo, tf, tlo, -tlo});   // slow in [tlo, -1]
            rects.push_back({tlo, tf, ns, thi + 1});  // slow in [ns, ns + thi]
            rects.push_back({tlo, -tlo, 0, ns});     // fast in [tlo, -1]
            rects.push_back({nf, thi + 1, 0, ns});   // fast in [nf, nf + thi]
        }
        for (const Rect& r : rects) {
            const int npen = r.fcnt * r.scnt;
            if (npen <= 0) continue;
            // the packed fields (check_table bounds the edges so that they fit)
            if (r.flo < -512 || r.flo > 511 || r.slo < -512 || r.slo > 511 || r.fcnt > 2047) {
                if (bad) *bad = true;
                return {};
            }
            const int code = (r.flo + 512) | ((r.slo + 512) << 10) | (r.fcnt << 20);
            for (int p0 = 0; p0 < npen; p0 += W)
                items.push_back(WorkItem{p, p0, code, (p0 + W - 1 < npen - 1) ? p0 + W - 1 : npen - 1});
        }
    }
    return xcd_order(items);
}

// (Re)build a group's work lists for W pencils a block.
// (Re)build a group's work lists for W pencils a block; the lists they
// replace are freed.
int set_group_W(wmb_ctx* c, int d, int stage, SweepGroup& G, int W) {
    auto rebuild = [&](DevList& L, SweepPart part) -> int {
        bool bad = false;
        std::vector<WorkItem> items = sweep_items(c, d, G.n, G.tlo, G.thi, W < 0 ? (-W) % 512 : W, part, -1, &bad);
        if (bad) return fail(c, WMB_EINVAL, "sweep work list: pencil rectangle outside the packed range");
        WorkItem* nd = nullptr;
        int rc = upload(c, &nd, items);
        if (rc) return rc;
        release(c, L.d);
        L.d = nd;
        L.n = (int)items.size();
        return WMB_OK;
    };
    int rc = rebuild(G.wl, PART_ALL);
    if (c->ngroups > 1 && G.wlg.size() < (size_t)c->ngroups) G.wlg.resize(c->ngroups);
    for (int g = 0; g < c->ngroups && c->ngroups > 1 && !rc; g++) {
        std::vector<WorkItem> items = sweep_items(c, d, G.n, G.tlo, G.thi, W < 0 ? (-W) % 512 : W, PART_ALL, g);
        WorkItem* nd = nullptr;
        if (!items.empty() && (rc = upload(c, &nd, items))) break;
        release(c, G.wlg[g].d);
        G.wlg[g].d = nd;
        G.wlg[g].n = (int)items.size();
    }
    if (!rc && d == 0 && stage == 0) rc = rebuild(G.wl_in, PART_INTERIOR);
    if (!rc && d == 0 && stage == 0) rc = rebuild(G.wl_fr, PART_FRAME);
    if (rc) return rc;
    G.W = W;
    return WMB_OK;
}

// The fused x/y corrector (xy_rows > 0): for the patches whose x edge is n,
// one item a z-plane k in [-3, n_z + 2] (beyond [-1, n_z] the z predictor
// records only) and band of y-face rows, the rows [-1, n_y + 2) cut into
// near-equal bands of at most rb rows.  Planes outermost, so that
// consecutive blocks of a patch share the z-flux plane between them.
std::vector<WorkItem> xy_items(const wmb_ctx* c, int n, int rb, int group = -1) {
    std::vector<WorkItem> items;
    for (int p = 0; p < c->npatch; p++) {
        if (c->desc[p].n[0] != n || !in_plan(c, p)) continue;
        if (group >= 0 && c->pgroup[p] != group) continue;
        const int* e = c->desc[p].n;
        const int E = e[1] + 3, nb = (E + rb - 1) / rb;
        for (int k = -3; k <= e[2] + 2; k++)
            for (int b = 0; b < nb; b++) {
                const int y0 = -1 + E * b / nb, y1 = -1 + E * (b + 1) / nb;
                items.push_back(WorkItem{p, k + XY_BIAS, (y0 + XY_BIAS) | ((y1 + XY_BIAS) << 16), 0});
            }
    }
    return xcd_order(items);
}

// rows of the fused corrector's block for x edge n: the largest band of any
// patch of that edge (frozen or absent ones too, so that the launch shape
// does not change when the plan does) plus the limiter's three halo rows
int xy_rt(const wmb_ctx* c, int n, int rb) {
    int rt = 0;
    for (int p = 0; p < c->npatch; p++) {
        if (c->desc[p].n[0] != n) continue;
        const int E = c->desc[p].n[1] + 3, nb = (E + rb - 1) / rb;
        rt = std::max(rt, (E + nb - 1) / nb + 3);
    }
    return rt;
}

// whether bands of at most rb rows fit the fused corrector's blocks for
// every x edge (1024 threads, 64 KiB of LDS)
bool xy_ok(const wmb_ctx* c, int rb) {
    if (rb < 1 || rb > 64) return false;
    for (const auto& G : c->sweeps[0][1]) {
        const long long t = (long long)G.P * xy_rt(c, G.n, rb);
        if (t > 1024 || (long long)c->esize * 16 * t > 64 * 1024) return false;
    }
    return true;
}

// Switch the fused x/y corrector off (rb = 0) or on with bands of at most rb
// rows: (re)build its lists, freeing the ones they replace.
int set_xy(wmb_ctx* c, int rb) {
    for (auto& G : c->sweeps[0][1]) {
        release(c, G.wxy.d);
        G.wxy = DevList{};
        for (auto& L : G.wxyg) {
            release(c, L.d);
            L = DevList{};
        }
        G.RT = 0;
        if (rb <= 0) continue;
        std::vector<WorkItem> items = xy_items(c, G.n, rb);
        G.wxy.n = (int)items.size();
        int rc = upload(c, &G.wxy.d, items);
        if (rc) return rc;
        if (c->ngroups > 1 && G.wxyg.size() < (size_t)c->ngroups) G.wxyg.resize(c->ngroups);
        for (int g = 0; g < c->ngroups && c->ngroups > 1; g++) {
            std::vector<WorkItem> gi = xy_items(c, G.n, rb, g);
            G.wxyg[g].n = (int)gi.size();
            if (!gi.empty() && (rc = upload(c, &G.wxyg[g].d, gi))) return rc;
        }
        G.RT = xy_rt(c, G.n, rb);
    }
    c->xy_rows = rb > 0 ? rb : 0;
    return WMB_OK;
}

int build_sweeps(wmb_ctx* c) {
    for (int d = 0; d < 3; d++) {
        for (int stage = 0; stage < 2; stage++) {
            const int zlo = stage == 0 ? -4 : -3;
            const int extra = stage == 0 ? 8 : 6;
            const int tlo = stage == 0 ? -3 : -1, thi = stage == 0 ? 2 : 0;
            // group patches by their edge along d (same pencil length)
            std::vector<int> sizes;
            for (int p = 0; p < c->npatch; p++) {
                int n = c->desc[p].n[d];
                bool seen = false;
                for (int s : sizes) seen |= (s == n);
                if (!seen) sizes.push_back(n);
            }
            for (int n : sizes) {
                SweepGroup G;
                G.P = n + extra;
                G.zlo = zlo;
                G.tlo = tlo;
                G.thi = thi;
                G.n = n;
                int rc = set_group_W(c, d, stage, G, choose_W(d, G.P, c->esize));
                if (rc) return rc;
                c->sweeps[d][stage].push_back(G);
            }
        }
    }
    return WMB_OK;
}

void free_graphs(wmb_ctx* c) {
    // the launch stream's completion does not mean every parallel branch of
    // a replayed graph has retired: destroying the executable before the
    // whole device is idle keeps the memory its kernels used from ever being
    // freed (measured on ROCm 7: a pool freed after wmb_destroy stayed
    // allocated unless the device was synchronised first)
    if (c->gexec[0] || c->gexec[1]) (void)hipDeviceSynchronize();  // teardown: nothing to report
    for (int i = 0; i < 2; i++) {
        if (c->gexec[i]) (void)hipGraphExecDestroy(c->gexec[i]);  // teardown: nothing to report
        if (c->graph[i]) (void)hipGraphDestroy(c->graph[i]);
        c->gexec[i] = nullptr;
        c->graph[i] = nullptr;
    }
}

// Plan the stage work lists again for the current active set (after a
// freeze, thaw, removal or addition), in place: a list whose items still fit
// its buffer keeps the buffer and its length (the rest padded with empty
// items, whose blocks exit at once), so the captured graphs, which hold the
// buffers and the grid sizes, stay valid.  Only a list that outgrows its
// buffer (a thaw after the tiles were re-planned smaller) is reallocated,
// and then the graphs are captured again.  Dropping the inactive patches'
// items keeps the blocks that run spread over the CUs: where a launch's
// blocks are all resident at once (the 512-zone Steps 8-11 tiles at 32^3),
// a checkerboard of frozen patches otherwise left every fourth pair of
// block ids, and with them whole CUs, without work.
int replan(wmb_ctx* c) {
    c->plan_dirty = false;
    CKH(hipStreamSynchronize(c->stream));  // no launch in flight reads the lists
    bool regrid = false;
    auto put = [&](DevList& L, std::vector<WorkItem> items) -> int {
        if (L.d && items.size() <= (size_t)L.n) {
            items.resize((size_t)L.n, WorkItem{-1, 0, 0, 0});
            if (L.n > 0) CKH(hipMemcpy(L.d, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice));
            return WMB_OK;
        }
        release(c, L.d);
        L = DevList{};
        regrid = true;
        L.n = (int)items.size();
        return upload(c, &L.d, items);
    };
    int rc = WMB_OK;
    for (int d = 0; d < 3 && !rc; d++)
        for (int stage = 0; stage < 2 && !rc; stage++)
            for (auto& G : c->sweeps[d][stage]) {
                const int W = G.W < 0 ? (-G.W) % 512 : G.W;
                if (!rc) rc = put(G.wl, sweep_items(c, d, G.n, G.tlo, G.thi, W, PART_ALL));
                for (int g = 0; g < c->ngroups && c->ngroups > 1 && !rc; g++)
                    rc = put(G.wlg[g], sweep_items(c, d, G.n, G.tlo, G.thi, W, PART_ALL, g));
                if (!rc && d == 0 && stage == 0) rc = put(G.wl_in, sweep_items(c, d, G.n, G.tlo, G.thi, W, PART_INTERIOR));
                if (!rc && d == 0 && stage == 0) rc = put(G.wl_fr, sweep_items(c, d, G.n, G.tlo, G.thi, W, PART_FRAME));
            }
    for (auto& G : c->sweeps[0][1]) {
        if (c->xy_rows <= 0) break;
        if (!rc) rc = put(G.wxy, xy_items(c, G.n, c->xy_rows));
        for (int g = 0; g < c->ngroups && c->ngroups > 1 && !rc; g++)
            rc = put(G.wxyg[g], xy_items(c, G.n, c->xy_rows, g));
    }
    const std::vector<int> rows = x_rows(c);
    if (!rc) rc = put(c->wl_cth, tile_items(c, -2, 2, -2, 2, c->cth_tx, 256, nullptr));
    if (!rc) rc = put(c->wl_upd, upd_items(c, c->upd_zones, &rows));
    for (int g = 0; g < c->ngroups && c->ngroups > 1 && !rc; g++) {
        rc = put(c->wl_cth_g[g], tile_items(c, -2, 2, -2, 2, c->cth_tx, 256, nullptr, g));
        if (!rc) rc = put(c->wl_upd_g[g], upd_items(c, c->upd_zones, &rows, g));
    }
    if (regrid) free_graphs(c);
    return rc;
}


// One graph per state copy: fill ghosts, dt = cfl / smax, step (whose final
// update refills smax for the next replay).  Replays require smax to hold the
// current state's maximum at their start.
int capture_graphs(wmb_ctx* c) {
    // nothing runs during capture: the host-side state flags are restored
    const int saved_state = c->smax_state;
    const bool saved_xg = c->xg_valid, saved_kept = c->edges_kept;
    const int cur_start = c->cur;
    auto restore = [&]() {
        c->cur = cur_start;
        c->smax_state = saved_state;
        c->xg_valid = saved_xg;
        c->edges_kept = saved_kept;
    };
    for (int k = 0; k < 2; k++) {
        const int cur0 = c->cur;
        CKH(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
        // grouped schedule: the exchange first, on the main stream; else the
        // exchange on its own branch beside the interior x sweep
        int rc = c->ngroups > 1 ? dispatch_fill(c, FILL_YZ) : fork_fill_yz(c);
        if (!rc) rc = run_finalize(c);
        if (!rc) rc = dispatch_step(c, true);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->stream, &g);
        if (rc || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            restore();
            return rc ? rc : fail(c, WMB_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        }
        c->graph[cur0] = g;
        e = hipGraphInstantiate(&c->gexec[cur0], g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            restore();
            return fail(c, WMB_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        // dispatch_step flipped cur; the second capture covers the other copy
    }
    restore();
    return WMB_OK;
}

template <typename R>
void to_device_layout(const double* src, R* dst, const PatchDev& P, int g, size_t n3) {
    (void)n3;
    for (int k = 0; k < P.n[2]; k++)
        for (int j = 0; j < P.n[1]; j++)
            for (int i = 0; i < P.n[0]; i++) {
                size_t s = ((size_t)k * P.n[1] + j) * P.n[0] + i;
                size_t d = ((size_t)(k + g) * P.N[1] + (j + g)) * P.N[0] + (i + g);
                dst[d] = (R)src[s];
            }
}

template <typename R>
void from_device_layout(const R* src, double* dst, const PatchDev& P, int g) {
    for (int k = 0; k < P.n[2]; k++)
        for (int j = 0; j < P.n[1]; j++)
            for (int i = 0; i < P.n[0]; i++) {
                size_t d = ((size_t)k * P.n[1] + j) * P.n[0] + i;
                size_t s = ((size_t)(k + g) * P.N[1] + (j + g)) * P.N[0] + (i + g);
                dst[d] = (double)src[s];
            }
}

template <typename R>
int set_state_t(wmb_ctx* c, int ip, const double* q, const double* b) {
    const PatchDev& P = c->hpatch[ip];
    const int g = c->p.ghost;
    const size_t n3 = (size_t)P.n[0] * P.n[1] * P.n[2];
    // validate: finite, rho > 0, P > 0
    for (size_t t = 0; t < n3; t++) {
        double u[8];
        for (int k = 0; k < 8; k++) {
            u[k] = q[k * n3 + t];
            if (!std::isfinite(u[k])) return fail(c, WMB_ESTATE, "non-finite q");
        }
        for (int k = 0; k < 3; k++)
            if (!std::isfinite(b[k * n3 + t])) return fail(c, WMB_ESTATE, "non-finite b");
        if (!(u[0] > 0.0)) return fail(c, WMB_ESTATE, "rho <= 0");
        double pr = (c->p.gamma - 1.0) * (u[7] - 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0] -
                                          0.5 * (u[4] * u[4] + u[5] * u[5] + u[6] * u[6]));
        if (!(pr > 0.0)) return fail(c, WMB_ESTATE, "pressure <= 0");
    }
    // the 11 arrays of a state copy are contiguous in the patch region: one
    // host image (ghosts NaN until the next exchange), one copy
    std::vector<R> img((size_t)11 * P.vol, (R)NAN);
    R* base = (R*)c->pool + P.base + (long long)(c->cur ? F_ST1 : F_ST0) * P.vol;
    if (c->smax_state != SMAX_ZERO) c->smax_state = SMAX_DIRTY;
    for (int f = 0; f < 11; f++) {
        const double* src = f < 8 ? q + f * n3 : b + (f - 8) * n3;
        R* buf = img.data() + (size_t)f * P.vol;
        to_device_layout<R>(src, buf, P, g, n3);
        const int a = f - 8;
        if (a >= 0 && P.nb[2 * a + 1] < 0) {
            // the patch owns its right face along an axis that ends at a domain
            // boundary: it starts as a copy of the face to its left
            const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
            const long long st = a == 0 ? 1LL : (a == 1 ? (long long)P.N[0] : (long long)P.N[0] * P.N[1]);
            for (int t2 = 0; t2 < P.n[a2]; t2++)
                for (int t1 = 0; t1 < P.n[a1]; t1++) {
                    int c3[3];
                    c3[a] = g + P.n[a];
                    c3[a1] = g + t1;
                    c3[a2] = g + t2;
                    const long long x = ((long long)c3[2] * P.N[1] + c3[1]) * P.N[0] + c3[0];
                    buf[(size_t)x] = buf[(size_t)(x - st)];
                }
        }
    }
    CKH(hipMemcpyAsync(base, img.data(), sizeof(R) * img.size(), hipMemcpyHostToDevice, c->stream));
    CKH(hipStreamSynchronize(c->stream));
    return WMB_OK;
}

template <typename R>
int get_state_t(wmb_ctx* c, int ip, double* q, double* b, bool stored) {
    const PatchDev& P = c->hpatch[ip];
    const int g = c->p.ghost;
    const size_t n3 = (size_t)P.n[0] * P.n[1] * P.n[2];
    std::vector<R> img((size_t)11 * P.vol);
    const R* base = (const R*)c->pool + P.base + (long long)(c->cur ? F_ST1 : F_ST0) * P.vol;
    CKH(hipMemcpyAsync(img.data(), base, sizeof(R) * img.size(), hipMemcpyDeviceToHost, c->stream));
    CKH(hipStreamSynchronize(c->stream));
    for (int f = 0; f < 11; f++) {
        double* dst = f < 8 ? q : b;
        if (!dst) continue;
        const R* buf = img.data() + (size_t)f * P.vol;
        int ff = f < 8 ? f : f - 8;
        if (stored) {
            for (long long t = 0; t < P.vol; t++) dst[(size_t)ff * P.vol + t] = (double)buf[t];
        } else {
            from_device_layout<R>(buf, dst + (size_t)ff * n3, P, g);
        }
    }
    return WMB_OK;
}

template <typename R>
int debug_stage_t(wmb_ctx* c, int ip, int stage, double* out) {
    const PatchDev& P = c->hpatch[ip];
    const long long V = P.vol;
    std::vector<R> buf((size_t)V);
    auto fetch = [&](int slot) -> int {  // a slot of the step's intermediates
        CKH(hipMemcpyAsync(buf.data(), (const R*)c->pool + P.sbase + (long long)slot * V, sizeof(R) * V,
                           hipMemcpyDeviceToHost, c->stream));
        CKH(hipStreamSynchronize(c->stream));
        return WMB_OK;
    };
    if (stage == 1 || stage == 5) {
        const int fs = stage == 1 ? F_FL1 : F_FL2;
        for (int d = 0; d < 3; d++) {
            int rowlab[7] = {0, 1, 2, 3, 7, 4 + (d + 1) % 3, 4 + (d + 2) % 3};
            for (long long t = 0; t < V; t++) out[((size_t)d * 8 + 4 + d) * V + t] = 0.0;
            for (int r = 0; r < 7; r++) {
                int rc = fetch(fs + 7 * d + r);
                if (rc) return rc;
                for (long long t = 0; t < V; t++) out[((size_t)d * 8 + rowlab[r]) * V + t] = (double)buf[t];
            }
        }
        return WMB_OK;
    }
    int slot = stage == 3 ? F_BH : (stage == 6 ? F_ED : -1);
    if (slot < 0) return fail(c, WMB_EINVAL, "stage not kept after the step (2: Step-3 edges are overwritten by Step 9)");
    if (stage == 6 && !c->edges_kept) return fail(c, WMB_ESTATE, "Step-9 edges are stored only by steps run with wmb_keep_stages on");
    for (int k = 0; k < 3; k++) {
        int rc = fetch(slot + k);
        if (rc) return rc;
        for (long long t = 0; t < V; t++) out[(size_t)k * V + t] = (double)buf[t];
    }
    return WMB_OK;
}

// Diagnostics on the device (compensated sums, fixed reduction order) into
// the 12 doubles at out: totals[8], max normalised div b, max |div b|, floor
// activations, protected faces.  rec holds wl_diag.n records.
template <typename R>
int enqueue_diag(wmb_ctx* c, double* rec, double* out) {
    const double dmin = std::fmin(c->p.dx[0], std::fmin(c->p.dx[1], c->p.dx[2]));
    hipError_t e = launch_diag<R>(c->pool, c->d_patch, c->wl_diag.d, c->wl_diag.n, c->dp, c->cur, rec, c->d_nfloor,
                                  (double)c->nzones, dmin, out, c->stream);
    if (e != hipSuccess) return fail_static(c, WMB_EHIP, "diagnostics: kernel launch failed");
    return WMB_OK;
}

template <typename R>
int diagnostics_t(wmb_ctx* c, double totals[8], double* dn, double* dr, int64_t* nfl, int64_t* npr) {
    int rc = enqueue_diag<R>(c, c->d_partial, c->d_diag_out);
    if (rc) return rc;
    double o[12];
    CKH(hipMemcpyAsync(o, c->d_diag_out, sizeof(o), hipMemcpyDeviceToHost, c->stream));
    CKH(hipStreamSynchronize(c->stream));
    if (totals)
        for (int k = 0; k < 8; k++) totals[k] = o[k];
    if (dn) *dn = o[8];
    if (dr) *dr = o[9];
    if (nfl) *nfl = (int64_t)o[10];
    if (npr) *npr = (int64_t)o[11];
    return WMB_OK;
}

// Sweep block shape search.  The pencil count per block W changes only the
// grouping of pencils into blocks, never the arithmetic of a face, so results
// are bitwise independent of the choice.  Timed on the current state: ghosts
// are refreshed and dt formed, then every candidate of each sweep group is
// launched (writing only step intermediates); the fastest W is kept.
template <typename R>
int autotune_t(wmb_ctx* c, int reps) {
    int rc = dispatch_fill(c);
    if (!rc) rc = ensure_smax(c);
    if (!rc) rc = run_finalize(c);
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    WorkItem* dl = nullptr;  // the candidate list of one timing
    WorkItem* tl = nullptr;  // a candidate tile list (library-owned)
    // every exit below goes through cleanup
    auto cleanup = [&](int code) -> int {
        if (dl) (void)hipFree(dl);
        if (tl) release(c, tl);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return code;
    };
#define CKT(call)                                                                                       \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return cleanup(fail(c, WMB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)));        \
    } while (0)
    CKT(hipEventCreate(&e0));
    CKT(hipEventCreate(&e1));
    const size_t es = sizeof(R);
    // the separate sweeps are timed first; the fused x/y corrector after them
    if (c->xy_rows > 0) {
        int rc0 = set_xy(c, 0);
        if (rc0) return cleanup(rc0);
    }
    for (int stage = 0; stage < 2; stage++) {
        if (stage == 1) {
            // intermediates the corrector sweeps read: Step-1 fluxes, edges, b^{n+1/2}
            hipError_t e = hipSuccess;
            for (int d = 0; d < 3 && e == hipSuccess; d++)
                for (auto& G : c->sweeps[d][0])
                    e = launch_group<R>(c, d, 1, G, G.wl, c->cur, c->d_nfloor + 2, c->stream);
            if (e == hipSuccess)
                e = launch_ct_half<R>(c->pool, c->d_patch, c->wl_cth.d, c->wl_cth.n, coef<R>(c), c->p.ghost, c->cur,
                                      c->d_sc, c->stream);
            if (e != hipSuccess) return cleanup(fail(c, WMB_EHIP, std::string("autotune: ") + hipGetErrorString(e)));
        }
        for (int d = 0; d < 3; d++) {
            for (auto& G : c->sweeps[d][stage]) {
                std::vector<int> cand;
                // pencil counts around the 64-lane wave: 5, 10 and 20 pencils
                // of 38 zones fill whole waves to 99%
                const int opts_x[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24};
                // negative: the marching form (beyond -512: loads one zone ahead)
                const int opts_t[] = {2, 4, 8, 16, 32, -64, -128, -256, -576, -640, -768};
                if (d == 0)
                    for (int W : opts_x) cand.push_back(W);
                else
                    for (int W : opts_t) cand.push_back(W);
                float best = 1e30f, bestp = 1e30f, bestm = 1e30f;
                int bestW = G.W;
                std::vector<std::pair<float, int>> timed;  // (ms, shape) of every candidate
                for (int W : cand) {
                    if (!shape_ok(d, G.P, es, W, stage + 1) || (W > 0 && G.P * W < 64)) continue;
                    std::vector<WorkItem> items = sweep_items(c, d, G.n, G.tlo, G.thi, W < 0 ? (-W) % 512 : W);
                    if (items.empty()) continue;
                    CKT(hipMalloc(&dl, sizeof(WorkItem) * items.size()));
                    CKT(hipMemcpy(dl, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice));
                    float tot = 1e30f;  // the fastest of the timed launches
                    hipError_t e = hipSuccess;
                    for (int r = 0; r <= reps && e == hipSuccess; r++) {
                        CKT(hipEventRecord(e0, c->stream));
                        SweepGroup T = G;
                        T.W = W;
                        e = launch_group<R>(c, d, stage + 1, T, DevList{dl, (int)items.size()}, c->cur, c->d_nfloor + 2,
                                            c->stream);
                        CKT(hipEventRecord(e1, c->stream));
                        CKT(hipEventSynchronize(e1));
                        float t = 0.f;
                        CKT(hipEventElapsedTime(&t, e0, e1));
                        if (r > 0) tot = std::min(tot, t);  // first launch is a warm-up
                    }
                    (void)hipFree(dl);
                    dl = nullptr;
                    if (e != hipSuccess)
                        return cleanup(fail(c, WMB_EHIP, std::string("autotune: ") + hipGetErrorString(e)));
                    if (tot < best) {
                        best = tot;
                        bestW = W;
                    }
                    if (W > 0 && tot < bestp) bestp = tot, G.Wp = W;
                    if (W < 0 && tot < bestm) bestm = tot, G.Wm = W;
                    timed.emplace_back(tot, W);
                }
                std::sort(timed.begin(), timed.end());
                G.Wx[0] = timed.size() > 1 ? timed[1].second : 0;
                G.Wx[1] = timed.size() > 2 ? timed[2].second : 0;
                if (bestW != G.W) {
                    int rc2 = set_group_W(c, d, stage, G, bestW);
                    if (rc2) return cleanup(rc2);
                }
            }
        }
    }
    // The graph runs the three sweeps of a stage concurrently, so the shapes
    // that are fastest alone need not be the fastest together: time whole
    // steps replayed from a captured graph for the shapes picked alone, then,
    // stage by stage, for each x group its second and third shapes alone,
    // then for the best pencil shapes and for the best marching shapes of
    // the y and z groups, keeping the fastest each time.  time_stage: a
    // whole step captured and replayed as a graph, as wmb_run_steps runs it
    // (the sweeps of a stage as branches), its results going nowhere the
    // next step reads: the update writes the other state copy, floors,
    // protected faces and the signal-speed maximum go to the sinks, and the
    // current copy and the flags are restored
    auto time_stage = [&](float* ms) -> int {
        unsigned long long *smax0 = c->d_smax, *nfl0 = c->d_nfloor;
        const int cur0 = c->cur, ss0 = c->smax_state;
        const bool xg0 = c->xg_valid, ek0 = c->edges_kept;
        c->d_smax = smax0 + 2;
        c->d_nfloor = nfl0 + 2;
        hipGraph_t gr = nullptr;
        hipGraphExec_t ge = nullptr;
        int rc4 = WMB_OK;
        hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed);
        if (e == hipSuccess) {
            e = hipEventRecord(c->ev_join, c->stream);  // the exchange is done
            if (e == hipSuccess) rc4 = run_step<R>(c, true);
            hipError_t e2 = hipStreamEndCapture(c->stream, &gr);
            if (e == hipSuccess) e = e2;
        }
        c->d_smax = smax0;
        c->d_nfloor = nfl0;
        c->cur = cur0;
        c->smax_state = ss0;
        c->xg_valid = xg0;
        c->edges_kept = ek0;
        if (!rc4 && e == hipSuccess) e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
        float tot = 1e30f;
        for (int r = 0; r <= reps && !rc4 && e == hipSuccess; r++) {
            e = hipEventRecord(e0, c->stream);
            if (e == hipSuccess) e = hipGraphLaunch(ge, c->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (r > 0) tot = std::min(tot, t);
        }
        // a graph executable is destroyed only on an idle device (ROCm 7
        // otherwise keeps the memory its kernels used from being freed)
        (void)hipDeviceSynchronize();
        if (ge) (void)hipGraphExecDestroy(ge);
        if (gr) (void)hipGraphDestroy(gr);
        if (rc4) return cleanup(rc4);
        if (e != hipSuccess) return cleanup(fail(c, WMB_EHIP, std::string("autotune: ") + hipGetErrorString(e)));
        *ms = tot;
        return WMB_OK;
    };
    for (int stage = 0; stage < 2; stage++) {
        float best = 0.f;
        int rc2 = time_stage(&best);
        if (rc2) return rc2;
        // the x sweeps: the second and third shapes alone, one group at a time
        for (auto& G : c->sweeps[0][stage])
            for (int a = 0; a < 2; a++) {
                const int W0 = G.W, W1 = G.Wx[a];
                if (W1 == 0 || W1 == W0) continue;
                if ((rc2 = set_group_W(c, 0, stage, G, W1))) return cleanup(rc2);
                float t = 0.f;
                if ((rc2 = time_stage(&t))) return rc2;
                if (t < best) {
                    best = t;
                } else if ((rc2 = set_group_W(c, 0, stage, G, W0))) {
                    return cleanup(rc2);
                }
            }
        std::vector<int> alone;
        for (int d = 1; d < 3; d++)
            for (auto& G : c->sweeps[d][stage]) alone.push_back(G.W);
        int choice = 0;  // 0: alone, 1: all pencil, 2: all marching
        for (int alt = 1; alt <= 2; alt++) {
            bool differs = false, valid = true;
            for (int d = 1; d < 3; d++)
                for (auto& G : c->sweeps[d][stage]) {
                    const int W = alt == 1 ? G.Wp : G.Wm;
                    valid = valid && W != 0;
                    differs = differs || W != G.W;
                }
            if (!valid || !differs) continue;
            for (int d = 1; d < 3 && !rc2; d++)
                for (auto& G : c->sweeps[d][stage])
                    if (!rc2) rc2 = set_group_W(c, d, stage, G, alt == 1 ? G.Wp : G.Wm);
            if (rc2) return cleanup(rc2);
            float t = 0.f;
            if ((rc2 = time_stage(&t))) return rc2;
            if (t < best) {
                best = t;
                choice = alt;
            }
            // back to the alone shapes before the next alternative
            size_t k = 0;
            for (int d = 1; d < 3 && !rc2; d++)
                for (auto& G : c->sweeps[d][stage])
                    if (!rc2) rc2 = set_group_W(c, d, stage, G, alone[k++]);
            if (rc2) return cleanup(rc2);
        }
        if (choice)
            for (int d = 1; d < 3 && !rc2; d++)
                for (auto& G : c->sweeps[d][stage])
                    if (!rc2) rc2 = set_group_W(c, d, stage, G, choice == 1 ? G.Wp : G.Wm);
        if (rc2) return cleanup(rc2);
    }
    // The fused x/y corrector: bands of 6, 9, 12 or 18 rows, each with the z
    // corrector (then reading the stored records) as marching sweeps of 256
    // or 64 pencils a block or pencil sweeps of 16, against the separate
    // sweeps as chosen above; whole steps replayed as a graph.
    {
        float best = 0.f;
        int rc2 = time_stage(&best);
        if (rc2) return rc2;
        int best_rb = 0;
        std::vector<int> zw, best_zw;
        for (auto& G : c->sweeps[2][1]) zw.push_back(G.W);
        best_zw = zw;
        for (int rb : {6, 9, 12, 18}) {
            if (!xy_ok(c, rb)) continue;
            if ((rc2 = set_xy(c, rb))) return cleanup(rc2);
            for (int W : {-256, -64, 16}) {
                std::vector<int> cur_zw;
                for (auto& G : c->sweeps[2][1]) {
                    const int w = shape_ok(2, G.P, es, W, 2) ? W : G.W;
                    if (w != G.W && (rc2 = set_group_W(c, 2, 1, G, w))) return cleanup(rc2);
                    cur_zw.push_back(w);
                }
                float t = 0.f;
                if ((rc2 = time_stage(&t))) return rc2;
                if (t < best) best = t, best_rb = rb, best_zw = cur_zw;
            }
        }
        if ((rc2 = set_xy(c, best_rb))) return cleanup(rc2);
        size_t i = 0;
        for (auto& G : c->sweeps[2][1]) {
            const int w = best_zw[i++];
            if (w != G.W && (rc2 = set_group_W(c, 2, 1, G, w))) return cleanup(rc2);
        }
    }
    // The tiles of Steps 3-4 (widest tile along x) and of Steps 8-11 (zones
    // a tile plane): time each candidate's whole launch.  The intermediates
    // they read are those the stage-2 timings left; the update writes only
    // the other state copy (and the x-ghosts there), its floor count and
    // signal-speed maximum go to the sinks, so nothing the next step reads
    // changes.
    {
        const std::vector<int> rows = x_rows(c);
        auto time_tiles = [&](int kind, int v, float* ms) -> int {
            DevList L;
            // kind 0: Steps 3-4; 1: Steps 8-11, one block a tile; 2: the same on the queues
            int rc3 = kind == 0 ? build_tile_list(c, -2, 2, -2, 2, v, 256, nullptr, L)
                                : build_upd_list(c, v, &rows, L);
            if (rc3) return cleanup(rc3);
            tl = L.d;  // released by cleanup on an error exit
            hipError_t e = hipSuccess;
            float tot = 1e30f;
            for (int r = 0; r <= reps && e == hipSuccess; r++) {
                CKT(hipEventRecord(e0, c->stream));
                e = kind == 0 ? launch_ct_half<R>(c->pool, c->d_patch, L.d, L.n, coef<R>(c), c->p.ghost, c->cur, c->d_sc,
                                                  c->stream)
                              : launch_update<R>(c->pool, c->d_patch, L.d, L.n, c->dp, coef<R>(c), c->cur, c->d_sc,
                                                 c->d_nfloor + 2, c->d_smax + 2, 0, v, kind == 2 ? c->d_queue : nullptr,
                                                 c->stream);
                CKT(hipEventRecord(e1, c->stream));
                CKT(hipEventSynchronize(e1));
                float t = 0.f;
                CKT(hipEventElapsedTime(&t, e0, e1));
                if (r > 0) tot = std::min(tot, t);
            }
            if (e != hipSuccess) return cleanup(fail(c, WMB_EHIP, std::string("autotune: ") + hipGetErrorString(e)));
            tl = nullptr;
            release(c, L.d);
            *ms = tot;
            return WMB_OK;
        };
        const int cth_opts[] = {40, 20, 13};
        const int upd_opts[] = {256, upd_tile_zones_max((int)es)};
        int best_tx = c->cth_tx, best_z = c->upd_zones, best_q = c->upd_queue;
        float bt = 1e30f, bz = 1e30f;
        for (int v : cth_opts) {
            float t = 0.f;
            int rc3 = time_tiles(0, v, &t);
            if (rc3) return rc3;
            if (t < bt) bt = t, best_tx = v;
        }
        for (int q = 0; q < 2; q++)
            for (int k = 0; k < 2; k++) {
                if (k == 1 && upd_opts[1] == upd_opts[0]) break;
                float t = 0.f;
                int rc3 = time_tiles(1 + q, upd_opts[k], &t);
                if (rc3) return rc3;
                if (t < bz) bz = t, best_z = upd_opts[k], best_q = q;
            }
        c->upd_queue = best_q;
        if (best_tx != c->cth_tx || best_z != c->upd_zones) {
            c->cth_tx = best_tx;
            c->upd_zones = best_z;
            int rc3 = build_ct_update_lists(c);
            if (rc3) return cleanup(rc3);
        }
    }
#undef CKT
    free_graphs(c);  // launch plans changed
    return cleanup(WMB_OK);
}

// Autotune choices kept for the life of the process, keyed by what decides
// the timings: the device architecture, the precision, the ghost width, the
// limiter and protection variants of the sweeps, and the patch extents with
// their counts.  A value is the quadruples wmb_autotune reports.
std::mutex tune_mu;
std::vector<std::pair<std::string, std::vector<int32_t>>> tune_cache;

std::string tune_key(const wmb_ctx* c) {
    hipDeviceProp_t prop;
    std::string arch = hipGetDeviceProperties(&prop, c->device) == hipSuccess ? prop.gcnArchName : "?";
    std::vector<std::string> ext;
    for (const auto& d : c->desc)
        ext.push_back(std::to_string(d.n[0]) + "x" + std::to_string(d.n[1]) + "x" + std::to_string(d.n[2]));
    std::sort(ext.begin(), ext.end());
    std::string key = arch + "|" + std::to_string(c->esize) + "|" + std::to_string(c->p.ghost) + "|" +
                      (c->p.limiter_beta == 1.0 ? "mm" : "sweby") + "|" +
                      ((c->p.rho_protect > 0.0 || c->p.p_protect > 0.0) ? "prot" : "plain");
    for (size_t i = 0; i < ext.size();) {
        size_t j = i;
        while (j < ext.size() && ext[j] == ext[i]) j++;
        key += "|" + ext[i] + "*" + std::to_string(j - i);
        i = j;
    }
    return key;
}

std::vector<int32_t> tuning_quads(const wmb_ctx* c) {
    std::vector<int32_t> q;
    for (int stage = 0; stage < 2; stage++)
        for (int d = 0; d < 3; d++)
            for (const auto& G : c->sweeps[d][stage]) q.insert(q.end(), {stage + 1, d, G.n, G.W});
    q.insert(q.end(), {3, 0, 0, c->cth_tx});
    q.insert(q.end(), {4, 0, 0, c->upd_zones});
    q.insert(q.end(), {5, 0, 0, c->upd_queue});
    q.insert(q.end(), {6, 0, 0, c->xy_rows});
    return q;
}

// ---------------------------------------------------------------------------
// Static records of the allocation-free diagnostics (wmb_diagnostics_noalloc):
// NOALLOC_RECORDS records of DIAG_REC doubles (5 MiB) in a device array that
// every GPU the library runs on holds until the process ends.  In host code
// the array's name is only a stand-in: kernels get the device address that
// hipGetSymbolAddress returns for the current device, taken once per device
// when a context is bound to it (wmb_init_patches).
// ---------------------------------------------------------------------------
constexpr int NOALLOC_RECORDS = 32768;
static __device__ __align__(256) double scratch[NOALLOC_RECORDS * DIAG_REC];

constexpr int MAX_DEVICES = 64;
double* scratch_dev[MAX_DEVICES] = {};
std::mutex scratch_mu;

// Side streams of the step graphs, borrowed from a per-device pool and given
// back (never destroyed) when a context ends.  On ROCm 7, destroying a stream
// that took part in a graph capture before the memory its captured kernels
// used is freed keeps that memory from ever being freed, and the caller
// frees its pool only after wmb_destroy.
std::vector<hipStream_t> spare_streams[MAX_DEVICES];
std::mutex stream_mu;

int borrow_stream(wmb_ctx* c, hipStream_t* out) {
    int dev = -1;
    CKH(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail_static(c, WMB_EHIP, "device index beyond the stream table");
    {
        std::lock_guard<std::mutex> lk(stream_mu);
        if (!spare_streams[dev].empty()) {
            *out = spare_streams[dev].back();
            spare_streams[dev].pop_back();
            return WMB_OK;
        }
    }
    CKH(hipStreamCreateWithFlags(out, hipStreamNonBlocking));
    return WMB_OK;
}

void return_stream(int dev, hipStream_t s) {
    if (!s) return;
    (void)hipStreamSynchronize(s);  // teardown: nothing to report
    if (dev < 0 || dev >= MAX_DEVICES) return;
    std::lock_guard<std::mutex> lk(stream_mu);
    spare_streams[dev].push_back(s);
}

int bind_scratch(wmb_ctx* c) {
    int dev = -1;
    CKH(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail_static(c, WMB_EHIP, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[dev]) {
        void* p = nullptr;
        CKH(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        scratch_dev[dev] = static_cast<double*>(p);
    }
    c->noalloc_rec = scratch_dev[dev];
    return WMB_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

// Patch groups of the step: pgroup from deal_rows, the group lists, and for
// concurrent groups (not serial) a stream and an event per group
int apply_groups(wmb_ctx* c, int groups) {
    free_graphs(c);
    if (groups > 1) {
        c->pgroup = deal_rows(c->npatch, c->desc.data(), groups);
        for (int g = 1; g < groups && !c->serial; g++) {
            if (!c->gstream[g]) {
                int rc = borrow_stream(c, &c->gstream[g]);
                if (rc) return rc;
            }
            if (!c->ev_g[g]) CKH(hipEventCreateWithFlags(&c->ev_g[g], hipEventDisableTiming));
        }
    }
    c->ngroups = groups;
    if (groups == 1) return WMB_OK;
    for (int d = 0; d < 3; d++)
        for (int stage = 0; stage < 2; stage++)
            for (auto& SG : c->sweeps[d][stage]) {
                int rc = set_group_W(c, d, stage, SG, SG.W);
                if (rc) return rc;
            }
    if (c->xy_rows > 0) {
        int rc = set_xy(c, c->xy_rows);
        if (rc) return rc;
    }
    return build_ct_update_lists(c);
}

extern "C" {

int wmb_create(const wmb_params* p, wmb_ctx** out) {
    if (!out) return WMB_EINVAL;
    *out = nullptr;
    int rc = check_params(p);
    if (rc) return rc;
    wmb_ctx* c = new (std::nothrow) wmb_ctx();
    if (!c) return WMB_ENOMEM;
    c->err.reserve(256);  // fixed messages fit without a later allocation
    c->p = *p;
    c->esize = esize_of(p);
    c->dp.gamma = p->gamma;
    c->dp.cfl = p->cfl;
    for (int k = 0; k < 7; k++) c->dp.eps[k] = p->eps[k];
    make_coef(*p, c->cf32);
    make_coef(*p, c->cf64);
    c->dp.limiter_beta = p->limiter_beta;
    c->dp.rho_floor = p->rho_floor;
    c->dp.p_floor = p->p_floor;
    for (int a = 0; a < 3; a++) c->dp.dx[a] = p->dx[a];
    c->dp.degen_tol = p->degen_tol;
    c->dp.ghost = p->ghost;
    c->dp.dt_lag = p->dt_lag;
    *out = c;
    return WMB_OK;
}

int wmb_pool_bytes(const wmb_params* p, int32_t npatch, const wmb_patch_desc* d, uint64_t* bytes) {
    if (check_params(p) || npatch <= 0 || !d || !bytes) return WMB_EINVAL;
    for (int i = 0; i < npatch; i++)
        for (int a = 0; a < 3; a++)
            if (d[i].n[a] < 1 || d[i].n[a] > max_edge(esize_of(p))) return WMB_EINVAL;
    *bytes = plan_pool(npatch, d, p->ghost, esize_of(p), p->scratch_groups).total;
    return WMB_OK;
}

int wmb_init_patches(wmb_ctx* c, int32_t npatch, const wmb_patch_desc* d, void* dev_pool, uint64_t pool_bytes,
                     void* hip_stream) {
    if (!c) return WMB_EINVAL;
    if (c->inited) return fail(c, WMB_EORDER, "patches already initialised");
    if (npatch <= 0 || !d || !dev_pool) return fail(c, WMB_EINVAL, "bad arguments");
    std::string why;
    if (check_table(npatch, d, c->p.ghost, c->esize, why)) return fail(c, WMB_EINVAL, why);
    uint64_t need = 0;
    wmb_pool_bytes(&c->p, npatch, d, &need);
    if (pool_bytes < need)
        return fail(c, WMB_ESIZE, "pool has " + std::to_string(pool_bytes) + " bytes, needs " + std::to_string(need));
    c->npatch = npatch;
    c->desc.assign(d, d + npatch);
    c->pool = dev_pool;
    c->pool_bytes = pool_bytes;
    CKH(hipGetDevice(&c->device));
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        int rco = borrow_stream(c, &c->stream);
        if (rco) return rco;
        c->own_stream = true;
    }
    int rcs = borrow_stream(c, &c->side);
    if (!rcs) rcs = borrow_stream(c, &c->side2);
    if (rcs) return rcs;
    CKH(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    CKH(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    for (auto& ev : c->ev_br) CKH(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    const int g = c->p.ghost;
    const PoolLayout lay = plan_pool(npatch, d, g, c->esize, c->p.scratch_groups);
    c->hpatch.resize(npatch);
    for (int i = 0; i < npatch; i++) {
        PatchDev& P = c->hpatch[i];
        for (int a = 0; a < 3; a++) {
            P.n[a] = d[i].n[a];
            P.N[a] = d[i].n[a] + 2 * g;
        }
        P.vol = vol_of(d[i], g);
        P.base = (long long)(lay.base[i] / c->esize);
        P.sbase = (long long)(lay.sbase[i] / c->esize);
        const int faces[6] = {12, 14, 10, 16, 4, 22};
        for (int t = 0; t < 6; t++) P.nb[t] = d[i].nbr[faces[t]];
        P.active = 1;
        P.present = 1;
    }
    int rc;
    if ((rc = upload(c, &c->d_patch, c->hpatch))) return rc;
    if ((rc = build_fill_lists(c))) return rc;
    if ((rc = build_box_list(c, BOX_INTERIOR, c->wl_int))) return rc;
    if ((rc = build_diag_list(c))) return rc;
    c->cth_tx = 40;
    c->upd_zones = choose_upd_zones(c);
    if ((rc = build_ct_update_lists(c))) return rc;
    c->nfrozen = 0;
    if ((rc = build_sweeps(c))) return rc;
    // FP32: the fused corrector with 9-row bands (6 where those blocks do not
    // fit), the fastest measured at 256^3; FP64 keeps the separate sweeps
    c->xy_rows = 0;
    if (c->esize == 4) {
        const int rb = xy_ok(c, 9) ? 9 : (xy_ok(c, 6) ? 6 : 0);
        if (rb && (rc = set_xy(c, rb))) return rc;
    }
    if (c->p.scratch_groups > 1) {
        c->serial = true;
        if ((rc = apply_groups(c, c->p.scratch_groups))) return rc;
    }
    // the signal-speed maxima of the current and the previous state, and a
    // sink for tuning runs
    if ((rc = dev_alloc(c, &c->d_smax, 3))) return rc;
    if ((rc = dev_alloc(c, &c->d_sc, 1))) return rc;
    // counters: floor activations, protected faces, and two sinks for tuning runs
    if ((rc = dev_alloc(c, &c->d_nfloor, 4))) return rc;
    if ((rc = dev_alloc(c, &c->d_queue, 64))) return rc;
    if ((rc = dev_alloc(c, &c->d_partial, (size_t)c->wl_diag.n * DIAG_REC))) return rc;
    if ((rc = dev_alloc(c, &c->d_diag_out, 12))) return rc;
    c->nzones = 0;
    for (int p = 0; p < npatch; p++) c->nzones += (long long)d[p].n[0] * d[p].n[1] * d[p].n[2];
    if ((rc = bind_scratch(c))) return rc;
    CKH(hipMemsetAsync(c->d_smax, 0, 3 * sizeof(unsigned long long), c->stream));
    CKH(hipMemsetAsync(c->d_sc, 0, sizeof(StepConst), c->stream));
    CKH(hipMemsetAsync(c->d_nfloor, 0, 4 * sizeof(unsigned long long), c->stream));
    CKH(hipMemsetAsync(c->d_queue, 0, 64 * sizeof(unsigned int), c->stream));
    CKH(hipStreamSynchronize(c->stream));
    c->cur = 0;
    c->smax_state = SMAX_ZERO;
    c->inited = true;
    return WMB_OK;
}

int freeze_sync(wmb_ctx* c, int patch);

int wmb_set_state(wmb_ctx* c, int32_t patch, const double* q, const double* b) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (patch < 0 || patch >= c->npatch || !q || !b) return fail(c, WMB_EINVAL, "bad patch or null array");
    c->xg_valid = false;  // the neighbours' x-ghosts of this patch are stale
    int rc = c->esize == 4 ? set_state_t<float>(c, patch, q, b) : set_state_t<double>(c, patch, q, b);
    if (!rc && c->hpatch[patch].present && !c->hpatch[patch].active) rc = freeze_sync(c, patch);
    return rc;
}

int wmb_get_state(wmb_ctx* c, int32_t patch, double* q, double* b) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (patch < 0 || patch >= c->npatch) return fail(c, WMB_EINVAL, "bad patch");
    return c->esize == 4 ? get_state_t<float>(c, patch, q, b, false) : get_state_t<double>(c, patch, q, b, false);
}

int wmb_get_stored(wmb_ctx* c, int32_t patch, double* q, double* b) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (patch < 0 || patch >= c->npatch) return fail(c, WMB_EINVAL, "bad patch");
    return c->esize == 4 ? get_state_t<float>(c, patch, q, b, true) : get_state_t<double>(c, patch, q, b, true);
}

int wmb_fill_ghosts(wmb_ctx* c) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    return dispatch_fill(c);
}

int wmb_compute_dt(wmb_ctx* c, double* dt_out) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    int rc = dispatch_dt(c);
    if (rc) return rc;
    if (dt_out) {
        CKH(hipMemcpyAsync(dt_out, &c->d_sc->dt, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        CKH(hipStreamSynchronize(c->stream));
    }
    return WMB_OK;
}

int wmb_advance(wmb_ctx* c, double dt) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (c->plan_dirty) {
        int rc = replan(c);
        if (rc) return rc;
    }
    if (dt > 0.0) {
        if (!std::isfinite(dt)) return fail(c, WMB_EINVAL, "non-finite dt");
        // the limit of the current state: an explicit reduction (the maximum
        // the last update folded in may be the lagged one under dt_lag)
        double lim = 0.0;
        int rc = c->esize == 4 ? run_reduce<float>(c) : run_reduce<double>(c);
        if (!rc) rc = wmb_compute_dt(c, &lim);
        if (rc) return rc;
        if (dt > lim * (1.0 + 1e-12)) return fail(c, WMB_ECFL, "dt above the CFL limit " + std::to_string(lim));
        CKH(launch_set_dt(c->d_sc, dt, c->dp, c->stream));
    }
    return dispatch_step(c);
}

int wmb_run_steps(wmb_ctx* c, int32_t nsteps) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (nsteps < 0) return fail(c, WMB_EINVAL, "nsteps < 0");
    if (nsteps == 0) return WMB_OK;
    if (c->plan_dirty) {
        int rc = replan(c);
        if (rc) return rc;
    }
    if (!c->gexec[0]) {
        int rc = capture_graphs(c);
        if (rc) {
            free_graphs(c);
            return rc;
        }
    }
    int rc = ensure_smax(c);
    if (!rc && !c->xg_valid) rc = dispatch_fill(c, FILL_X);  // the graphs start at the y pass
    if (rc) return rc;
    for (int s = 0; s < nsteps; s++) {
        CKH(hipGraphLaunch(c->gexec[c->cur], c->stream));
        c->cur ^= 1;
    }
    c->smax_state = SMAX_CLEAN;
    c->xg_valid = true;
    return WMB_OK;
}

int wmb_diagnostics(wmb_ctx* c, double totals[8], double* max_divb_norm, double* max_divb_raw, int64_t* n_floored,
                    int64_t* n_protected) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    return c->esize == 4 ? diagnostics_t<float>(c, totals, max_divb_norm, max_divb_raw, n_floored, n_protected)
                         : diagnostics_t<double>(c, totals, max_divb_norm, max_divb_raw, n_floored, n_protected);
}

int wmb_diagnostics_noalloc(wmb_ctx* c, double* dev_out) {
    if (!c) return WMB_EINVAL;
    if (!dev_out) return fail_static(c, WMB_EINVAL, "diagnostics_noalloc: null output");
    if (!c->inited) return fail_static(c, WMB_EORDER, "wmb_init_patches first");
    if (c->wl_diag.n > NOALLOC_RECORDS)
        return fail_static(c, WMB_ESIZE,
                           "diagnostics_noalloc: the batch needs more than 32768 records (one per started run of "
                           "32768 interior zones of a patch); use wmb_diagnostics");
    if (!c->noalloc_rec) return fail_static(c, WMB_EHIP, "diagnostics_noalloc: no scratch address for this device");
    return c->esize == 4 ? enqueue_diag<float>(c, c->noalloc_rec, dev_out) : enqueue_diag<double>(c, c->noalloc_rec, dev_out);
}

int wmb_debug_stage(wmb_ctx* c, int32_t patch, int32_t stage, double* out) {
    if (!c || !out) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (patch < 0 || patch >= c->npatch) return fail(c, WMB_EINVAL, "bad patch");
    return c->esize == 4 ? debug_stage_t<float>(c, patch, stage, out) : debug_stage_t<double>(c, patch, stage, out);
}

int wmb_autotune(wmb_ctx* c, int32_t reps, int32_t* chosen, int32_t nchosen) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (c->plan_dirty) {
        int rc = replan(c);
        if (rc) return rc;
    }
    const std::string key = tune_key(c);
    std::vector<int32_t> q;
    if (reps >= 0) {
        std::lock_guard<std::mutex> lk(tune_mu);
        for (const auto& kv : tune_cache)
            if (kv.first == key) q = kv.second;
    }
    if (!q.empty()) {
        int rc = wmb_set_tuning(c, q.data(), (int32_t)q.size());
        if (rc) return rc;
    } else {
        int r = reps < 0 ? -reps : reps;
        int rc = c->esize == 4 ? autotune_t<float>(c, r < 1 ? 1 : r) : autotune_t<double>(c, r < 1 ? 1 : r);
        if (rc) return rc;
        q = tuning_quads(c);
        std::lock_guard<std::mutex> lk(tune_mu);
        bool found = false;
        for (auto& kv : tune_cache)
            if (kv.first == key) kv.second = q, found = true;
        if (!found) tune_cache.emplace_back(key, q);
    }
    if (chosen) {
        int k = 0;
        for (int32_t v : q) {
            if (k >= nchosen) return WMB_OK;
            chosen[k++] = v;
        }
        if (k < nchosen) chosen[k] = 0;
    }
    return WMB_OK;
}

int wmb_set_tuning(wmb_ctx* c, const int32_t* quads, int32_t n) {
    if (!c || (!quads && n > 0) || n < 0 || n % 4) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    // check every entry before applying any
    for (int k = 0; k + 4 <= n; k += 4) {
        const int stage = quads[k], d = quads[k + 1], edge = quads[k + 2], W = quads[k + 3];
        if (stage == 5) {
            if (d != 0 || edge != 0 || (W != 0 && W != 1))
                return fail(c, WMB_EINVAL, "tuning entry: (5, 0, 0, 0 or 1) picks the Steps 8-11 launch");
            continue;
        }
        if (stage == 6) {
            if (d != 0 || edge != 0 || W < 0 || (W > 0 && !xy_ok(c, W)))
                return fail(c, WMB_EINVAL, "tuning entry: (6, 0, 0, r) fuses the x and y correctors with bands of at "
                                           "most r rows (0: separate), each block within 1024 threads and 64 KiB of LDS");
            continue;
        }
        if (stage == 3 || stage == 4) {
            if (d != 0 || edge != 0) return fail(c, WMB_EINVAL, "tuning entry: tile entries have axis 0 and edge 0");
            if (stage == 3 && (W < 4 || W > 40))
                return fail(c, WMB_EINVAL, "tuning entry: Steps 3-4 tiles are 4 to 40 zones wide");
            if (stage == 4 && W != 256 && W != upd_tile_zones_max((int)c->esize))
                return fail(c, WMB_EINVAL, "tuning entry: Steps 8-11 tiles hold 256 zones a plane (512 in FP32)");
            continue;
        }
        if (stage < 1 || stage > 2 || d < 0 || d > 2 || W == 0) return fail(c, WMB_EINVAL, "bad tuning entry");
        for (auto& G : c->sweeps[d][stage - 1])
            if (G.n == edge && !shape_ok(d, G.P, c->esize, W, stage))
                return fail(c, WMB_EINVAL, "tuning entry: the marching form serves y and z with at most 256 pencils "
                                           "a block; the pencil form must fit 1024 threads and 64 KiB of LDS");
    }
    bool tiles = false;
    for (int k = 0; k + 4 <= n; k += 4) {
        const int stage = quads[k], d = quads[k + 1], edge = quads[k + 2], W = quads[k + 3];
        if (stage == 5) {
            c->upd_queue = W;
            continue;
        }
        if (stage == 6) {
            if (W != c->xy_rows) {
                int rc = set_xy(c, W);
                if (rc) return rc;
            }
            continue;
        }
        if (stage == 3 || stage == 4) {
            int& v = stage == 3 ? c->cth_tx : c->upd_zones;
            tiles = tiles || v != W;
            v = W;
            continue;
        }
        for (auto& G : c->sweeps[d][stage - 1]) {
            if (G.n != edge) continue;
            int rc = set_group_W(c, d, stage - 1, G, W);
            if (rc) return rc;
        }
    }
    if (tiles) {
        int rc = build_ct_update_lists(c);
        if (rc) return rc;
    }
    free_graphs(c);
    return WMB_OK;
}

int wmb_set_schedule(wmb_ctx* c, int32_t groups) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (c->serial)
        return groups == c->ngroups ? WMB_OK
                                    : fail(c, WMB_EINVAL, "schedule: fixed to the scratch groups of the pool layout");
    if (groups < 1 || groups > 4) return fail(c, WMB_EINVAL, "schedule: 1 to 4 patch groups");
    if (groups == c->ngroups) return WMB_OK;
    return apply_groups(c, groups);
}

// A frozen patch reads the same in both state copies, ghosts included, so
// that its neighbours can pull from it whichever copy is current: refresh
// every ghost of the current copy, then copy the patch's whole stored box
// into the other one.
int freeze_sync(wmb_ctx* c, int patch) {
    const PatchDev& P = c->hpatch[patch];
    int rc = dispatch_fill(c, FILL_ALL);
    if (rc) return rc;
    const size_t bytes = (size_t)11 * P.vol * c->esize;
    char* pool = (char*)c->pool;
    const long long cur0 = (long long)(c->cur ? F_ST1 : F_ST0), oth0 = (long long)(c->cur ? F_ST0 : F_ST1);
    CKH(hipMemcpyAsync(pool + (P.base + oth0 * P.vol) * c->esize, pool + (P.base + cur0 * P.vol) * c->esize, bytes,
                       hipMemcpyDeviceToDevice, c->stream));
    return WMB_OK;
}

// the device copy of one patch-table entry, ordered on the library stream
int push_patch(wmb_ctx* c, int patch) {
    CKH(launch_set_patch(c->d_patch, patch, c->hpatch[patch], c->stream));
    return WMB_OK;
}

int wmb_set_active(wmb_ctx* c, int32_t patch, int32_t active) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (patch < 0 || patch >= c->npatch) return fail(c, WMB_EINVAL, "bad patch");
    PatchDev& P = c->hpatch[patch];
    if (!P.present) return fail(c, WMB_EORDER, "patch is absent (wmb_set_present)");
    const int on = active != 0;
    if (P.active == on) return WMB_OK;
    if (!on) {
        int rc = freeze_sync(c, patch);
        if (rc) return rc;
    }
    P.active = on;
    int rc = push_patch(c, patch);
    if (rc) return rc;
    c->nfrozen += on ? -1 : 1;
    c->plan_dirty = true;
    // the folded signal-speed maximum no longer covers the active set
    if (c->smax_state == SMAX_CLEAN) c->smax_state = SMAX_DIRTY;
    c->xg_valid = false;
    return WMB_OK;
}

// Face t of the patch table (-x, +x, -y, +y, -z, +z) in the init table's 27
// entries.
constexpr int kFaceEntry[6] = {12, 14, 10, 16, 4, 22};

int wmb_set_present(wmb_ctx* c, int32_t patch, int32_t present) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (patch < 0 || patch >= c->npatch) return fail(c, WMB_EINVAL, "bad patch");
    PatchDev& P = c->hpatch[patch];
    const int on = present != 0;
    if (P.present == on) return WMB_OK;
    std::vector<int> touched{patch};
    if (!on) {
        // bring every ghost and shared face up to date first (the faces the
        // slot shares with its neighbours keep these values and become the
        // neighbours' own boundary faces), and give both state copies the
        // slot's state, which it keeps while absent
        int rc = freeze_sync(c, patch);
        if (rc) return rc;
        if (!P.active) c->nfrozen--;
        for (int t = 0; t < 6; t++) {
            const int q = P.nb[t];
            if (q < 0) continue;
            PatchDev& Q = c->hpatch[q];
            if (Q.nb[t ^ 1] == patch) Q.nb[t ^ 1] = -1;
            touched.push_back(q);
            P.nb[t] = -1;
        }
        P.present = 0;
        P.active = 0;
    } else {
        // link to the init table's face neighbours that are present
        for (int t = 0; t < 6; t++) {
            const int q = c->desc[patch].nbr[kFaceEntry[t]];
            if (q < 0 || q == patch || !c->hpatch[q].present) continue;
            P.nb[t] = q;
            c->hpatch[q].nb[t ^ 1] = patch;
            touched.push_back(q);
        }
        // periodic with itself along an axis (one patch across): its own neighbour
        for (int t = 0; t < 6; t++)
            if (c->desc[patch].nbr[kFaceEntry[t]] == patch) P.nb[t] = patch;
        P.present = 1;
        P.active = 1;
    }
    for (int q : touched) {
        int rc = push_patch(c, q);
        if (rc) return rc;
    }
    c->nzones = 0;
    for (int p = 0; p < c->npatch; p++)
        if (c->hpatch[p].present) c->nzones += (long long)c->desc[p].n[0] * c->desc[p].n[1] * c->desc[p].n[2];
    if (c->smax_state == SMAX_CLEAN) c->smax_state = SMAX_DIRTY;
    c->xg_valid = false;
    c->plan_dirty = true;
    return WMB_OK;
}

int wmb_keep_stages(wmb_ctx* c, int32_t on) {
    if (!c) return WMB_EINVAL;
    if (c->keep_edges != (on != 0)) free_graphs(c);  // the update launch carries the flag
    c->keep_edges = on != 0;
    return WMB_OK;
}

int wmb_profile_step(wmb_ctx* c, double* ms, int32_t nclass) {
    if (!c || !ms) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (nclass < WMB_NCLASS) return fail(c, WMB_EINVAL, "ms must hold WMB_NCLASS entries");
    int rc = c->plan_dirty ? replan(c) : WMB_OK;
    if (!rc) rc = ensure_smax(c);
    if (!rc && !c->xg_valid) rc = dispatch_fill(c, FILL_X);  // as before a graph replay
    if (rc) return rc;
    // one event after every kernel class; with serial groups after every
    // class of every group (the fill and dt once), summed per class
    const int groups = (c->serial && c->ngroups > 1) ? c->ngroups : 1;
    const int nev = 2 + (WMB_NCLASS - 2) * groups;
    std::vector<hipEvent_t> ev(nev + 1, nullptr);
    for (auto& e : ev) CKH(hipEventCreate(&e));
    CKH(hipEventRecord(ev[0], c->stream));
    c->marks = ev.data() + 1;
    c->mark_cap = nev;
    c->nmark = 0;
    rc = dispatch_fill(c, FILL_YZ);
    if (!rc) rc = run_finalize(c);
    if (!rc) rc = dispatch_step(c);
    c->marks = nullptr;
    if (!rc && c->nmark != nev) rc = fail(c, WMB_EHIP, "profile: unexpected kernel count");
    if (!rc) {
        CKH(hipEventSynchronize(ev[nev]));
        for (int i = 0; i < WMB_NCLASS; i++) ms[i] = 0.0;
        for (int i = 0; i < nev; i++) {
            float t = 0.f;
            CKH(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
            ms[i < 2 ? i : 2 + (i - 2) % (WMB_NCLASS - 2)] += t;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return rc;
}

int wmb_destroy(wmb_ctx* c) {
    if (!c) return WMB_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);  // teardown: nothing to report
    free_graphs(c);
    for (void* p : c->owned) (void)hipFree(p);
    for (hipStream_t sd : {c->side, c->side2}) return_stream(c->device, sd);
    for (int g = 1; g < 4; g++) {
        return_stream(c->device, c->gstream[g]);
        if (c->ev_g[g]) (void)hipEventDestroy(c->ev_g[g]);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    for (hipEvent_t ev : c->ev_br)
        if (ev) (void)hipEventDestroy(ev);
    if (c->own_stream) return_stream(c->device, c->stream);
    delete c;
    return WMB_OK;
}

const char* wmb_strerror(int code) {
    switch (code) {
    case WMB_OK: return "ok";
    case WMB_EINVAL: return "invalid argument";
    case WMB_ENOMEM: return "out of memory";
    case WMB_EHIP: return "HIP runtime error";
    case WMB_ESTATE: return "invalid state (non-finite, rho <= 0 or P <= 0)";
    case WMB_ECFL: return "dt above the CFL limit";
    case WMB_ESIZE: return "device pool too small";
    case WMB_EORDER: return "call out of sequence";
    default: return "unknown error";
    }
}

const char* wmb_last_error(const wmb_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
