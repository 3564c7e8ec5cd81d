// wmb_runtime.hip -- host runtime behind the C ABI of include/wmb.h: context,
// patch tables, launch plans (work lists), ghost-exchange plan, dt and
// diagnostics plumbing, HIP-graph capture of one step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/wmb.h"
#include "wmb_internal.h"

namespace wmb {
template <typename R> hipError_t launch_fill(void*, const PatchDev*, const FillRegion*, int, int, hipStream_t);
template <typename R> hipError_t launch_dt(void*, const PatchDev*, const WorkItem*, int, const DevParams&, int, unsigned long long*, double*, hipStream_t);
template <typename R> hipError_t launch_emf_ref(void*, const PatchDev*, const WorkItem*, int, const DevParams&, int, Box, hipStream_t);
template <typename R> hipError_t launch_emf_half(void*, const PatchDev*, const WorkItem*, int, const DevParams&, int, const double*, Box, hipStream_t);
template <typename R> hipError_t launch_edge(void*, const PatchDev*, const WorkItem*, int, const DevParams&, int, Box, EdgeRanges, hipStream_t);
template <typename R> hipError_t launch_ct_half(void*, const PatchDev*, const WorkItem*, int, const DevParams&, int, const double*, Box, hipStream_t);
template <typename R> hipError_t launch_final(void*, const PatchDev*, const WorkItem*, int, const DevParams&, int, const double*, unsigned long long*, hipStream_t);
template <typename R> hipError_t launch_sweep(int, int, void*, const PatchDev*, const WorkItem*, int, const DevParams&, int, const double*, int, int, int, hipStream_t);
template <typename R> hipError_t launch_diag(const void*, const PatchDev*, const WorkItem*, int, const DevParams&, int, double*, hipStream_t);
}  // namespace wmb

using namespace wmb;

namespace {

struct DevList {
    WorkItem* d = nullptr;
    int n = 0;
};

struct SweepGroup {
    int P, W, zlo;
    DevList wl;
};

// Box of each box kernel, interior-relative [lo, n + hi]
const Box BOX_INTERIOR{0, -1};
const Box BOX_ER1{-3, 2};
const Box BOX_EDGE1{-2, 2};
const Box BOX_CTH{-2, 2};
const Box BOX_ER2{-1, 0};
const Box BOX_EDGE2{0, 0};

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
    int cur = 0;
    PatchDev* d_patch = nullptr;
    FillRegion* d_fill = nullptr;
    int nfill = 0;
    DevList wl_int, wl_er1, wl_edge1, wl_cth, wl_er2, wl_edge2;
    std::vector<SweepGroup> sweeps[3][2];
    unsigned long long* d_smax = nullptr;
    double* d_dt = nullptr;
    unsigned long long* d_nfloor = nullptr;
    double* d_partial = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    std::string err;
    std::vector<void*> owned;  // library-owned device allocations
    hipEvent_t* marks = nullptr;  // when set, an event is recorded after every kernel class
    int nmark = 0;
};

namespace {

int fail(wmb_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
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
    return WMB_OK;
}

size_t esize_of(const wmb_params* p) { return p->precision == WMB_FP32 ? 4 : 8; }

long long vol_of(const wmb_patch_desc& d, int g) {
    return (long long)(d.n[0] + 2 * g) * (d.n[1] + 2 * g) * (d.n[2] + 2 * g);
}

// per-patch region size in bytes, rounded to 256 B
uint64_t region_bytes(const wmb_patch_desc& d, int g, size_t es) {
    uint64_t b = (uint64_t)F_TOTAL * (uint64_t)vol_of(d, g) * es;
    return (b + 255) & ~uint64_t(255);
}

int check_table(int32_t np, const wmb_patch_desc* d, int g, std::string& why) {
    for (int i = 0; i < np; i++) {
        for (int a = 0; a < 3; a++)
            if (d[i].n[a] < g) {
                why = "patch " + std::to_string(i) + ": interior edge smaller than the ghost width";
                return WMB_EINVAL;
            }
        if (d[i].nbr[13] != i) {
            why = "patch " + std::to_string(i) + ": nbr[13] must be the patch itself";
            return WMB_EINVAL;
        }
        for (int t = 0; t < 27; t++) {
            int q = d[i].nbr[t];
            if (q < 0 || q >= np) {
                why = "patch " + std::to_string(i) + ": neighbour id out of range";
                return WMB_EINVAL;
            }
            int off[3] = {t % 3 - 1, (t / 3) % 3 - 1, t / 9 - 1};
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

void mark(wmb_ctx* c) {
    if (c->marks) hipEventRecord(c->marks[c->nmark++], c->stream);
}

template <typename R>
int run_fill(wmb_ctx* c) {
    hipError_t e = launch_fill<R>(c->pool, c->d_patch, c->d_fill, c->nfill, c->cur, c->stream);
    if (e != hipSuccess) return fail(c, WMB_EHIP, std::string("fill_ghosts: ") + hipGetErrorString(e));
    mark(c);
    return WMB_OK;
}

template <typename R>
int run_dt(wmb_ctx* c) {
    hipError_t e = launch_dt<R>(c->pool, c->d_patch, c->wl_int.d, c->wl_int.n, c->dp, c->cur, c->d_smax, c->d_dt, c->stream);
    if (e != hipSuccess) return fail(c, WMB_EHIP, std::string("dt_reduce: ") + hipGetErrorString(e));
    mark(c);
    return WMB_OK;
}

template <typename R>
int run_step(wmb_ctx* c) {
    hipError_t e;
    const int cur = c->cur;
#define STEPCK(what)                                                                        \
    if (e != hipSuccess) return fail(c, WMB_EHIP, std::string(what) + ": " + hipGetErrorString(e))
    e = launch_emf_ref<R>(c->pool, c->d_patch, c->wl_er1.d, c->wl_er1.n, c->dp, cur, BOX_ER1, c->stream);
    STEPCK("emf_ref");
    mark(c);
    for (int d = 0; d < 3; d++) {
        for (auto& G : c->sweeps[d][0]) {
            e = launch_sweep<R>(d, 1, c->pool, c->d_patch, G.wl.d, G.wl.n, c->dp, cur, c->d_dt, G.P, G.W, G.zlo, c->stream);
            STEPCK("sweep1");
        }
        mark(c);
    }
    e = launch_edge<R>(c->pool, c->d_patch, c->wl_edge1.d, c->wl_edge1.n, c->dp, F_FL1, BOX_EDGE1, EdgeRanges{-1, 0, -2, 2},
                       c->stream);
    STEPCK("edge_emf1");
    mark(c);
    e = launch_ct_half<R>(c->pool, c->d_patch, c->wl_cth.d, c->wl_cth.n, c->dp, cur, c->d_dt, BOX_CTH, c->stream);
    STEPCK("ct_half");
    mark(c);
    for (int d = 0; d < 3; d++) {
        for (auto& G : c->sweeps[d][1]) {
            e = launch_sweep<R>(d, 2, c->pool, c->d_patch, G.wl.d, G.wl.n, c->dp, cur, c->d_dt, G.P, G.W, G.zlo, c->stream);
            STEPCK("sweep2");
        }
        mark(c);
    }
    e = launch_emf_half<R>(c->pool, c->d_patch, c->wl_er2.d, c->wl_er2.n, c->dp, cur, c->d_dt, BOX_ER2, c->stream);
    STEPCK("emf_half");
    mark(c);
    e = launch_edge<R>(c->pool, c->d_patch, c->wl_edge2.d, c->wl_edge2.n, c->dp, F_FL2, BOX_EDGE2, EdgeRanges{0, -1, 0, 0},
                       c->stream);
    STEPCK("edge_emf2");
    mark(c);
    e = launch_final<R>(c->pool, c->d_patch, c->wl_int.d, c->wl_int.n, c->dp, cur, c->d_dt, c->d_nfloor, c->stream);
    STEPCK("final_update");
    mark(c);
#undef STEPCK
    c->cur ^= 1;
    return WMB_OK;
}

int dispatch_fill(wmb_ctx* c) { return c->esize == 4 ? run_fill<float>(c) : run_fill<double>(c); }
int dispatch_dt(wmb_ctx* c) { return c->esize == 4 ? run_dt<float>(c) : run_dt<double>(c); }
int dispatch_step(wmb_ctx* c) { return c->esize == 4 ? run_step<float>(c) : run_step<double>(c); }

int build_box_list(wmb_ctx* c, Box bx, DevList& out) {
    std::vector<WorkItem> items;
    for (int p = 0; p < c->npatch; p++) {
        long long e = 1;
        for (int a = 0; a < 3; a++) e *= (long long)(c->desc[p].n[a] + bx.hi - bx.lo + 1);
        int nb = (int)((e + 255) / 256);
        for (int b = 0; b < nb; b++) items.push_back(WorkItem{p, b, 0, 0});
    }
    out.n = (int)items.size();
    return upload(c, &out.d, items);
}

int choose_W(int d, int P, size_t es) {
    if (d == 0) {
        int W = 256 / P;
        return W < 1 ? 1 : W;
    }
    int W = 16;
    while (W > 1 && ((size_t)P * W > 1024 || es * 14 * (size_t)P * W > 64 * 1024)) W /= 2;
    return W;
}

int build_sweeps(wmb_ctx* c) {
    for (int d = 0; d < 3; d++) {
        const int FA = (d == 0) ? 1 : 0;
        const int SA = (d == 0) ? 2 : (d == 1 ? 2 : 1);
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
                G.W = choose_W(d, G.P, c->esize);
                std::vector<WorkItem> items;
                for (int p = 0; p < c->npatch; p++) {
                    if (c->desc[p].n[d] != n) continue;
                    int fhi = c->desc[p].n[FA] + thi, shi = c->desc[p].n[SA] + thi;
                    for (int sl = tlo; sl <= shi; sl++)
                        for (int f0 = tlo; f0 <= fhi; f0 += G.W)
                            items.push_back(WorkItem{p, f0, sl, (f0 + G.W - 1 < fhi) ? f0 + G.W - 1 : fhi});
                }
                G.wl.n = (int)items.size();
                int rc = upload(c, &G.wl.d, items);
                if (rc) return rc;
                c->sweeps[d][stage].push_back(G);
            }
        }
    }
    return WMB_OK;
}

int build_fill(wmb_ctx* c) {
    const int g = c->p.ghost;
    std::vector<FillRegion> regs;
    for (int i = 0; i < c->npatch; i++) {
        const wmb_patch_desc& D = c->desc[i];
        for (int t = 0; t < 27; t++) {
            if (t == 13) continue;
            int off[3] = {t % 3 - 1, (t / 3) % 3 - 1, t / 9 - 1};
            int q = D.nbr[t];
            const wmb_patch_desc& S = c->desc[q];
            FillRegion r;
            r.dst = i;
            r.src = q;
            for (int a = 0; a < 3; a++) {
                if (off[a] < 0) {
                    r.d0[a] = 0;
                    r.s0[a] = S.n[a];
                    r.ext[a] = g;
                } else if (off[a] > 0) {
                    r.d0[a] = g + D.n[a];
                    r.s0[a] = g;
                    r.ext[a] = g;
                } else {
                    r.d0[a] = g;
                    r.s0[a] = g;
                    r.ext[a] = D.n[a];
                }
            }
            regs.push_back(r);
        }
    }
    c->nfill = (int)regs.size();
    return upload(c, &c->d_fill, regs);
}

void free_graphs(wmb_ctx* c) {
    for (int i = 0; i < 2; i++) {
        if (c->gexec[i]) hipGraphExecDestroy(c->gexec[i]);
        if (c->graph[i]) hipGraphDestroy(c->graph[i]);
        c->gexec[i] = nullptr;
        c->graph[i] = nullptr;
    }
}

int capture_graphs(wmb_ctx* c) {
    for (int k = 0; k < 2; k++) {
        const int cur0 = c->cur;
        CKH(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
        int rc = dispatch_fill(c);
        if (!rc) rc = dispatch_dt(c);
        if (!rc) rc = dispatch_step(c);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->stream, &g);
        if (rc) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(c, WMB_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        c->graph[cur0] = g;
        CKH(hipGraphInstantiate(&c->gexec[cur0], g, nullptr, nullptr, 0));
        // dispatch_step flipped cur; the second capture covers the other copy
    }
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
    std::vector<R> buf((size_t)P.vol, (R)NAN);
    R* base = (R*)c->pool + P.base + (long long)(c->cur ? F_ST1 : F_ST0) * P.vol;
    for (int f = 0; f < 11; f++) {
        const double* src = f < 8 ? q + f * n3 : b + (f - 8) * n3;
        to_device_layout<R>(src, buf.data(), P, g, n3);
        CKH(hipMemcpyAsync(base + (long long)f * P.vol, buf.data(), sizeof(R) * P.vol, hipMemcpyHostToDevice, c->stream));
        CKH(hipStreamSynchronize(c->stream));
    }
    return WMB_OK;
}

template <typename R>
int get_state_t(wmb_ctx* c, int ip, double* q, double* b, bool stored) {
    const PatchDev& P = c->hpatch[ip];
    const int g = c->p.ghost;
    const size_t n3 = (size_t)P.n[0] * P.n[1] * P.n[2];
    std::vector<R> buf((size_t)P.vol);
    const R* base = (const R*)c->pool + P.base + (long long)(c->cur ? F_ST1 : F_ST0) * P.vol;
    for (int f = 0; f < 11; f++) {
        double* dst = f < 8 ? q : b;
        if (!dst) continue;
        CKH(hipMemcpyAsync(buf.data(), base + (long long)f * P.vol, sizeof(R) * P.vol, hipMemcpyDeviceToHost, c->stream));
        CKH(hipStreamSynchronize(c->stream));
        int ff = f < 8 ? f : f - 8;
        if (stored) {
            for (long long t = 0; t < P.vol; t++) dst[(size_t)ff * P.vol + t] = (double)buf[t];
        } else {
            from_device_layout<R>(buf.data(), dst + (size_t)ff * n3, P, g);
        }
    }
    return WMB_OK;
}

template <typename R>
int debug_stage_t(wmb_ctx* c, int ip, int stage, double* out) {
    const PatchDev& P = c->hpatch[ip];
    const long long V = P.vol;
    std::vector<R> buf((size_t)V);
    auto fetch = [&](int slot) -> int {
        CKH(hipMemcpyAsync(buf.data(), (const R*)c->pool + P.base + (long long)slot * V, sizeof(R) * V,
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
    for (int k = 0; k < 3; k++) {
        int rc = fetch(slot + k);
        if (rc) return rc;
        for (long long t = 0; t < V; t++) out[(size_t)k * V + t] = (double)buf[t];
    }
    return WMB_OK;
}

template <typename R>
int diagnostics_t(wmb_ctx* c, double totals[8], double* dn, double* dr, int64_t* nfl) {
    hipError_t e = launch_diag<R>(c->pool, c->d_patch, c->wl_int.d, c->wl_int.n, c->dp, c->cur, c->d_partial, c->stream);
    if (e != hipSuccess) return fail(c, WMB_EHIP, std::string("diag: ") + hipGetErrorString(e));
    std::vector<double> part((size_t)c->wl_int.n * 10);
    CKH(hipMemcpyAsync(part.data(), c->d_partial, sizeof(double) * part.size(), hipMemcpyDeviceToHost, c->stream));
    unsigned long long nf = 0;
    CKH(hipMemcpyAsync(&nf, c->d_nfloor, sizeof(nf), hipMemcpyDeviceToHost, c->stream));
    CKH(hipStreamSynchronize(c->stream));
    double sum[9] = {0}, comp[9] = {0}, mx = 0.0;
    for (int b = 0; b < c->wl_int.n; b++) {
        for (int k = 0; k < 9; k++) {
            double y = part[(size_t)b * 10 + k] - comp[k];
            double t = sum[k] + y;
            comp[k] = (t - sum[k]) - y;
            sum[k] = t;
        }
        mx = std::fmax(mx, part[(size_t)b * 10 + 9]);
    }
    long long nz = 0;
    for (int p = 0; p < c->npatch; p++) nz += (long long)c->desc[p].n[0] * c->desc[p].n[1] * c->desc[p].n[2];
    if (totals)
        for (int k = 0; k < 8; k++) totals[k] = sum[k];
    double brms = std::sqrt(sum[8] / (double)(nz ? nz : 1));
    if (brms < 1e-300) brms = 1e-300;
    double dmin = std::fmin(c->p.dx[0], std::fmin(c->p.dx[1], c->p.dx[2]));
    if (dr) *dr = mx;
    if (dn) *dn = mx * dmin / brms;
    if (nfl) *nfl = (int64_t)nf;
    return WMB_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

int wmb_create(const wmb_params* p, wmb_ctx** out) {
    if (!out) return WMB_EINVAL;
    *out = nullptr;
    int rc = check_params(p);
    if (rc) return rc;
    wmb_ctx* c = new (std::nothrow) wmb_ctx();
    if (!c) return WMB_ENOMEM;
    c->p = *p;
    c->esize = esize_of(p);
    c->dp.gamma = p->gamma;
    c->dp.cfl = p->cfl;
    for (int k = 0; k < 7; k++) c->dp.eps[k] = p->eps[k];
    c->dp.limiter_beta = p->limiter_beta;
    c->dp.rho_floor = p->rho_floor;
    c->dp.p_floor = p->p_floor;
    for (int a = 0; a < 3; a++) c->dp.dx[a] = p->dx[a];
    c->dp.degen_tol = p->degen_tol;
    c->dp.ghost = p->ghost;
    *out = c;
    return WMB_OK;
}

int wmb_pool_bytes(const wmb_params* p, int32_t npatch, const wmb_patch_desc* d, uint64_t* bytes) {
    if (check_params(p) || npatch <= 0 || !d || !bytes) return WMB_EINVAL;
    uint64_t tot = 0;
    for (int i = 0; i < npatch; i++) tot += region_bytes(d[i], p->ghost, esize_of(p));
    *bytes = tot;
    return WMB_OK;
}

int wmb_init_patches(wmb_ctx* c, int32_t npatch, const wmb_patch_desc* d, void* dev_pool, uint64_t pool_bytes,
                     void* hip_stream) {
    if (!c) return WMB_EINVAL;
    if (c->inited) return fail(c, WMB_EORDER, "patches already initialised");
    if (npatch <= 0 || !d || !dev_pool) return fail(c, WMB_EINVAL, "bad arguments");
    std::string why;
    if (check_table(npatch, d, c->p.ghost, why)) return fail(c, WMB_EINVAL, why);
    uint64_t need = 0;
    wmb_pool_bytes(&c->p, npatch, d, &need);
    if (pool_bytes < need)
        return fail(c, WMB_ESIZE, "pool has " + std::to_string(pool_bytes) + " bytes, needs " + std::to_string(need));
    c->npatch = npatch;
    c->desc.assign(d, d + npatch);
    c->pool = dev_pool;
    c->pool_bytes = pool_bytes;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        CKH(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    const int g = c->p.ghost;
    uint64_t off = 0;
    c->hpatch.resize(npatch);
    for (int i = 0; i < npatch; i++) {
        PatchDev& P = c->hpatch[i];
        for (int a = 0; a < 3; a++) {
            P.n[a] = d[i].n[a];
            P.N[a] = d[i].n[a] + 2 * g;
        }
        P.vol = vol_of(d[i], g);
        P.base = (long long)(off / c->esize);
        off += region_bytes(d[i], g, c->esize);
    }
    int rc;
    if ((rc = upload(c, &c->d_patch, c->hpatch))) return rc;
    if ((rc = build_fill(c))) return rc;
    if ((rc = build_box_list(c, BOX_INTERIOR, c->wl_int))) return rc;
    if ((rc = build_box_list(c, BOX_ER1, c->wl_er1))) return rc;
    if ((rc = build_box_list(c, BOX_EDGE1, c->wl_edge1))) return rc;
    if ((rc = build_box_list(c, BOX_CTH, c->wl_cth))) return rc;
    if ((rc = build_box_list(c, BOX_ER2, c->wl_er2))) return rc;
    if ((rc = build_box_list(c, BOX_EDGE2, c->wl_edge2))) return rc;
    if ((rc = build_sweeps(c))) return rc;
    if ((rc = dev_alloc(c, &c->d_smax, 1))) return rc;
    if ((rc = dev_alloc(c, &c->d_dt, 1))) return rc;
    if ((rc = dev_alloc(c, &c->d_nfloor, 1))) return rc;
    if ((rc = dev_alloc(c, &c->d_partial, (size_t)c->wl_int.n * 10))) return rc;
    CKH(hipMemsetAsync(c->d_smax, 0, sizeof(unsigned long long), c->stream));
    CKH(hipMemsetAsync(c->d_dt, 0, sizeof(double), c->stream));
    CKH(hipMemsetAsync(c->d_nfloor, 0, sizeof(unsigned long long), c->stream));
    CKH(hipStreamSynchronize(c->stream));
    c->cur = 0;
    c->inited = true;
    return WMB_OK;
}

int wmb_set_state(wmb_ctx* c, int32_t patch, const double* q, const double* b) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (patch < 0 || patch >= c->npatch || !q || !b) return fail(c, WMB_EINVAL, "bad patch or null array");
    return c->esize == 4 ? set_state_t<float>(c, patch, q, b) : set_state_t<double>(c, patch, q, b);
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
        CKH(hipMemcpyAsync(dt_out, c->d_dt, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        CKH(hipStreamSynchronize(c->stream));
    }
    return WMB_OK;
}

int wmb_advance(wmb_ctx* c, double dt) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (dt > 0.0) {
        if (!std::isfinite(dt)) return fail(c, WMB_EINVAL, "non-finite dt");
        double lim = 0.0;
        int rc = wmb_compute_dt(c, &lim);
        if (rc) return rc;
        if (dt > lim * (1.0 + 1e-12)) return fail(c, WMB_ECFL, "dt above the CFL limit " + std::to_string(lim));
        CKH(hipMemcpyAsync(c->d_dt, &dt, sizeof(double), hipMemcpyHostToDevice, c->stream));
        CKH(hipStreamSynchronize(c->stream));
    }
    return dispatch_step(c);
}

int wmb_run_steps(wmb_ctx* c, int32_t nsteps) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (nsteps < 0) return fail(c, WMB_EINVAL, "nsteps < 0");
    if (nsteps == 0) return WMB_OK;
    if (!c->gexec[0]) {
        int rc = capture_graphs(c);
        if (rc) {
            free_graphs(c);
            return rc;
        }
    }
    for (int s = 0; s < nsteps; s++) {
        CKH(hipGraphLaunch(c->gexec[c->cur], c->stream));
        c->cur ^= 1;
    }
    return WMB_OK;
}

int wmb_diagnostics(wmb_ctx* c, double totals[8], double* max_divb_norm, double* max_divb_raw, int64_t* n_floored) {
    if (!c) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    return c->esize == 4 ? diagnostics_t<float>(c, totals, max_divb_norm, max_divb_raw, n_floored)
                         : diagnostics_t<double>(c, totals, max_divb_norm, max_divb_raw, n_floored);
}

int wmb_debug_stage(wmb_ctx* c, int32_t patch, int32_t stage, double* out) {
    if (!c || !out) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (patch < 0 || patch >= c->npatch) return fail(c, WMB_EINVAL, "bad patch");
    return c->esize == 4 ? debug_stage_t<float>(c, patch, stage, out) : debug_stage_t<double>(c, patch, stage, out);
}

int wmb_profile_step(wmb_ctx* c, double* ms, int32_t nclass) {
    if (!c || !ms) return WMB_EINVAL;
    if (!c->inited) return fail(c, WMB_EORDER, "wmb_init_patches first");
    if (nclass < WMB_NCLASS) return fail(c, WMB_EINVAL, "ms must hold WMB_NCLASS entries");
    hipEvent_t ev[WMB_NCLASS + 1];
    for (int i = 0; i <= WMB_NCLASS; i++) CKH(hipEventCreate(&ev[i]));
    CKH(hipEventRecord(ev[0], c->stream));
    c->marks = ev + 1;
    c->nmark = 0;
    int rc = dispatch_fill(c);
    if (!rc) rc = dispatch_dt(c);
    if (!rc) rc = dispatch_step(c);
    c->marks = nullptr;
    if (!rc && c->nmark != WMB_NCLASS) rc = fail(c, WMB_EHIP, "profile: unexpected kernel count");
    if (!rc) {
        CKH(hipEventSynchronize(ev[WMB_NCLASS]));
        for (int i = 0; i < WMB_NCLASS; i++) {
            float t = 0.f;
            CKH(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
            ms[i] = t;
        }
    }
    for (int i = 0; i <= WMB_NCLASS; i++) hipEventDestroy(ev[i]);
    return rc;
}

int wmb_destroy(wmb_ctx* c) {
    if (!c) return WMB_OK;
    if (c->stream) hipStreamSynchronize(c->stream);
    free_graphs(c);
    for (void* p : c->owned) hipFree(p);
    if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
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
