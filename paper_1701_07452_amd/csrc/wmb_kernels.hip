// wmb_kernels.hip -- gfx950 kernels of one CTU+CT MHDTVD step over a batch of
// ghosted patches (Mendygral et al. 2017, Sect. 5.2 Steps 1-11, Appendix A).
//
// Every kernel is templated on the working precision R (float or double).
// The CFL reduction, floors and diagnostics are FP64 whatever R is.
//
// Kernel map (one step):
//   fill_pass<x,y,z>  ghost exchange in three dependent passes: x-ghosts of
//                     interior rows, then whole y-ghost rows, then whole
//                     z-ghost planes (each ghost value written once, rows and
//                     planes copied contiguously); after a step the x pass is
//                     already done by the update kernel
//   dt_reduce         FP64 max signal speed (only when no fused value exists)
//   dt_finalize       dt = cfl / smax, kept in device memory
//   sweep<d,1>        Step 1   MHDTVD fluxes from q^n, B_par = b^n    (hot);
//                              the x sweep also writes E^r (Step 2)
//   ct_half           Steps 3-4 fused, marching along z with the edge EMFs in
//                              LDS: b^{n+1/2} = b^n - dt/2 curl E
//   sweep<d,2>        Steps 5-7  transverse predictor + source, then MHDTVD
//                              fluxes with B_par = b^{n+1/2}        (hot)
//   update            Steps 8-11 fused, marching along z with E^r and the edge
//                              EMFs in LDS: q^{n+1}, b^{n+1}, zone field, FP64
//                              floors, and the FP64 signal-speed max of q^{n+1}
//                              for the next dt
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wmb_internal.h"

namespace wmb {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Reciprocal and square root: hardware v_rcp_f32 / v_sqrt_f32 (about 1 ulp)
// in the FP32 path, correctly rounded operations in the FP64 path.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double frsq(double x) { return 1.0 / sqrt(x); }
// smallest |alpha| divided by in the limiter's gamma (FP32: keeps the hardware
// reciprocal away from denormals; FP64: exact zero test)
__device__ __forceinline__ float alpha_min(float) { return 1e-30f; }
__device__ __forceinline__ double alpha_min(double) { return 0.0; }
// the limiter's gamma = dg / alpha.  FP64 divides: for a denormal alpha the
// reciprocal overflows to inf and 0 * inf would give NaN, while the quotient
// is finite (0 for dg = 0).  FP32 multiplies by the hardware reciprocal
// (alpha_min keeps alpha normal).
__device__ __forceinline__ float gdiv(float dg, float alpha) { return dg * frcp(alpha); }
__device__ __forceinline__ double gdiv(double dg, double alpha) { return dg / alpha; }

template <typename R>
__device__ __forceinline__ R sgn1(R x) { return x >= R(0) ? R(1) : R(-1); }

// The arithmetic helpers of the sweeps form fused multiply-adds only within
// a source expression (contract(on)), so that the pencil and the marching
// form of a sweep, which inline them into different code, round every face
// identically.

// coefficient of numerical viscosity Q_k(chi) (Appendix A); q4e = 1/(4 eps)
template <typename R>
__device__ __forceinline__ R qvisc(R chi, R eps, R q4e) {
#pragma clang fp contract(on)
    R ac = fabs(chi);
    if (ac < R(2) * eps) return chi * chi * q4e + eps;
    return ac;
}

// g_i = SIGN(gp) * SWEBY(gp, gm) (Appendix A), Sweby family with parameter
// beta; MM: beta = 1 (minmod), where both arguments of the outer max agree
// exactly and one branch is dropped.  Minmod is the median of gp, gm and 0,
// one v_med3_f32 in FP32 (the same value; a zero result may differ in sign,
// which no sum or product of the flux carries into a nonzero value).
template <bool MM, typename R>
__device__ __forceinline__ R sweby(R gp, R gm, R beta) {
#pragma clang fp contract(on)
    if constexpr (MM && sizeof(R) == 4) return __builtin_amdgcn_fmed3f(gp, gm, 0.0f);
    R s = sgn1(gp);
    if (MM) return s * fmax(R(0), fmin(fabs(gp), s * gm));
    R t1 = fmin(beta * fabs(gp), s * gm);
    R t2 = fmin(fabs(gp), beta * s * gm);
    return s * fmax(R(0), fmax(t1, t2));
}

template <typename R>
__device__ __forceinline__ R minmod2(R a, R b) {
#pragma clang fp contract(on)
    if (a > R(0) && b > R(0)) return fmin(a, b);
    if (a < R(0) && b < R(0)) return fmax(a, b);
    return R(0);
}

// per-step constants in the working precision
__device__ __forceinline__ float sc_dt(const StepConst& s, float) { return s.fdt; }
__device__ __forceinline__ double sc_dt(const StepConst& s, double) { return s.dt; }
__device__ __forceinline__ float sc_hdt(const StepConst& s, float) { return s.fhdt; }
__device__ __forceinline__ double sc_hdt(const StepConst& s, double) { return s.hdt; }
__device__ __forceinline__ float sc_lam(const StepConst& s, int d, float) { return s.flam[d]; }
__device__ __forceinline__ double sc_lam(const StepConst& s, int d, double) { return s.lam[d]; }
__device__ __forceinline__ float sc_il(const StepConst& s, int d, float) { return s.fil[d]; }
__device__ __forceinline__ double sc_il(const StepConst& s, int d, double) { return s.il[d]; }

// Raw buffer access to one patch region: SGPR descriptor, 32-bit VGPR byte
// offset of the zone, SGPR byte offset of the field (and of a neighbour
// shift), so no per-load 64-bit address arithmetic is spent.
constexpr int BUF_DWORD3 = 0x00020000;  // raw dword buffer, gfx9-family format
__device__ __forceinline__ __amdgpu_buffer_rsrc_t patch_rsrc(void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, BUF_DWORD3);
}
__device__ __forceinline__ float bload(float, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ double bload(double, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, 0);
}

__device__ __forceinline__ long long sidx(const PatchDev& P, int i, int j, int k) {
    return ((long long)k * P.N[1] + j) * P.N[0] + i;
}

__device__ __forceinline__ long long stride_of(const PatchDev& P, int a) {
    return a == 0 ? 1LL : (a == 1 ? (long long)P.N[0] : (long long)P.N[0] * P.N[1]);
}

// FP64 floors on one zone (density raised with momentum kept, then pressure
// raised by adding thermal energy).  Returns true if a floor fired.
template <typename R>
__device__ __forceinline__ bool apply_floor64(R u[8], const DevParams& p) {
#pragma clang fp contract(on)
    bool hit = false;
    double rho = (double)u[0];
    if (rho < p.rho_floor) {
        rho = p.rho_floor;
        u[0] = (R)rho;
        hit = true;
    }
    double m2 = (double)u[1] * u[1] + (double)u[2] * u[2] + (double)u[3] * u[3];
    double b2 = (double)u[4] * u[4] + (double)u[5] * u[5] + (double)u[6] * u[6];
    double pr = (p.gamma - 1.0) * ((double)u[7] - 0.5 * m2 / rho - 0.5 * b2);
    if (pr < p.p_floor) {
        u[7] = (R)((double)u[7] + (p.p_floor - pr) / (p.gamma - 1.0));
        hit = true;
    }
    return hit;
}

// The FP64 decision is the reference; in FP32 a zone whose FP32 pressure is
// above the floor by more than a bound on its FP32 rounding error (and whose
// density is above twice the floor) cannot be floored in FP64 either, so the
// FP64 evaluation is skipped for it.
__device__ __forceinline__ bool apply_floor(double u[8], const DevParams& p, const Coef<double>&) {
#pragma clang fp contract(on)
    return apply_floor64(u, p);
}
__device__ __forceinline__ bool apply_floor(float u[8], const DevParams& p, const Coef<float>& cf) {
#pragma clang fp contract(on)
    if (u[0] > 2.0f * cf.rho_floor) {
        float ir = frcp(u[0]);
        float ke = 0.5f * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) * ir;
        float me = 0.5f * (u[4] * u[4] + u[5] * u[5] + u[6] * u[6]);
        float pr = cf.gm1 * (u[7] - ke - me);
        float err = 1e-6f * cf.gm1 * (fabsf(u[7]) + ke + me);
        if (pr - err > cf.p_floor) return false;
    }
    return apply_floor64(u, p);
}

// ---------------------------------------------------------------------------
// box-kernel indexing: block (patch, blk) covers blockDim consecutive linear
// indices of an (ex, ey, ez) box, x fastest
// ---------------------------------------------------------------------------

struct BoxPos {
    int i, j, k;
    bool valid;
};

__device__ __forceinline__ BoxPos lin_pos(int blk, int ex, int ey, int ez) {
    int t = blk * blockDim.x + threadIdx.x;
    BoxPos r;
    r.valid = t < ex * ey * ez;
    r.i = t % ex;
    int u = t / ex;
    r.j = u % ey;
    r.k = u / ey;
    return r;
}

// interior-relative position in the box [lo, n+hi]^3
__device__ __forceinline__ BoxPos box_pos(const PatchDev& P, int blk, Box bx) {
    BoxPos r = lin_pos(blk, P.n[0] + bx.hi - bx.lo + 1, P.n[1] + bx.hi - bx.lo + 1, P.n[2] + bx.hi - bx.lo + 1);
    r.i += bx.lo;
    r.j += bx.lo;
    r.k += bx.lo;
    return r;
}

// ---------------------------------------------------------------------------
// ghost exchange, pass AX (0: x-ghosts of interior rows; 1: whole y-ghost rows
// of interior z-planes; 2: whole z-ghost planes).  Each pass copies from the
// face neighbour's interior (and, for passes 1-2, the ghosts the previous
// passes filled there), so edge and corner ghosts arrive through the chain
// x -> y -> z.  Bitwise copies of all 11 fields.
// ---------------------------------------------------------------------------

template <typename R, int AX>
__global__ void __launch_bounds__(256) fill_pass_kernel(R* __restrict__ pool, const PatchDev* __restrict__ patches,
                                                        const WorkItem* __restrict__ work, int g, int cur) {
    const WorkItem w = work[blockIdx.x];
    if (w.patch < 0) return;  // padding item (whole block)
    const PatchDev D = patches[w.patch];
    if (!D.present) return;  // absent slot
    // along a later pass's axis that ends at a domain boundary on the right,
    // the rows reach the boundary face n the patch owns: that later pass
    // copies the normal face there onto itself, so it must be in place
    const int wy = D.nb[3] < 0, wz = D.nb[5] < 0;
    int ex, ey, ez;
    if (AX == 0) {
        ex = 2 * g;
        ey = D.n[1] + wy;
        ez = D.n[2] + wz;
    } else if (AX == 1) {
        ex = D.N[0];
        ey = 2 * g;
        ez = D.n[2] + wz;
    } else {
        ex = D.N[0];
        ey = D.N[1];
        ez = 2 * g;
    }
    BoxPos p = lin_pos(w.a, ex, ey, ez);
    if (!p.valid) return;
    int d[3], s[3];
    int side;
    if (AX == 0) {
        side = p.i >= g;
        d[0] = side ? D.n[0] + p.i : p.i;  // p.i in [g, 2g) -> g + n + (p.i - g)
        d[1] = p.j + g;
        d[2] = p.k + g;
    } else if (AX == 1) {
        side = p.j >= g;
        d[0] = p.i;
        d[1] = side ? D.n[1] + p.j : p.j;
        d[2] = p.k + g;
    } else {
        side = p.k >= g;
        d[0] = p.i;
        d[1] = p.j;
        d[2] = side ? D.n[2] + p.k : p.k;
    }
    // a domain boundary (no neighbour, -1): zero-gradient extension from the
    // patch itself, the normal face field from the boundary face it owns
    const int nbq = D.nb[2 * AX + side];
    const bool wall = nbq < 0;
    const PatchDev S = wall ? D : patches[nbq];
    s[0] = d[0];
    s[1] = d[1];
    s[2] = d[2];
    // left ghost r = d - g < 0 comes from the neighbour's r + n_src; right ghost
    // r >= n_dst from the neighbour's r - n_dst
    s[AX] = wall ? (side ? g + D.n[AX] - 1 : g) : (side ? d[AX] - D.n[AX] : d[AX] + S.n[AX]);
    const long long di = sidx(D, d[0], d[1], d[2]);
    const long long si = sidx(S, s[0], s[1], s[2]);
    const long long sif = wall && side ? si + stride_of(D, AX) : si;  // boundary face n for b_AX
    R* dbase = pool + D.base + (long long)(cur ? F_ST1 : F_ST0) * D.vol;
    const R* sbase = pool + S.base + (long long)(cur ? F_ST1 : F_ST0) * S.vol;
#pragma unroll
    for (int c = 0; c < 11; c++)
        dbase[(long long)c * D.vol + di] = sbase[(long long)c * S.vol + (c == 8 + AX ? sif : si)];
}

// ---------------------------------------------------------------------------
// CFL signal speed (FP64): max_d (|v_d| + c_f,d) / dx_d, c_f,d the fast speed
// (Sect. 5) with B_d as the longitudinal field
// ---------------------------------------------------------------------------

__device__ __forceinline__ double signal_speed(const double u[8], const DevParams& p) {
    // the plain formula, operation for operation and without contraction,
    // so that the maximum (and dt) is the one the plain evaluation gives
#pragma clang fp contract(off)
    const double rho = u[0];
    const double v[3] = {u[1] / rho, u[2] / rho, u[3] / rho};
    const double b2 = u[4] * u[4] + u[5] * u[5] + u[6] * u[6];
    double pr = (p.gamma - 1.0) * (u[7] - 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - 0.5 * b2);
    if (pr < p.p_floor) pr = p.p_floor;
    const double a2 = p.gamma * pr / rho;
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double bd = u[4 + d];
        const double ca2 = bd * bd / rho;
        const double bp2 = (b2 - bd * bd) / rho;
        const double dpr = a2 - ca2 - bp2;
        const double dd = sqrt(dpr * dpr + 4.0 * a2 * bp2);
        const double cf = sqrt(0.5 * (a2 + ca2 + bp2 + dd));
        const double sd = (fabs(v[d]) + cf) / p.dx[d];
        if (sd > s) s = sd;
    }
    return s;
}

__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// block max (every thread of a block of at most 1024 threads must call) + atomicMax
__device__ __forceinline__ void block_max_atomic(double s, unsigned long long* smax_bits) {
    __shared__ double red[16];
    s = wave_max(s);
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int t = 1; t < (int)(blockDim.x >> 6); t++) m = fmax(m, red[t]);
        // positive doubles order like their bit patterns
        atomicMax(smax_bits, (unsigned long long)__double_as_longlong(m));
    }
}

template <typename R>
__global__ void __launch_bounds__(256) dt_reduce_kernel(const R* __restrict__ pool, const PatchDev* __restrict__ patches,
                                                        const WorkItem* __restrict__ work, DevParams prm, int cur,
                                                        unsigned long long* __restrict__ smax_bits) {
    const WorkItem w = work[blockIdx.x];
    if (w.patch < 0) return;  // padding item (whole block)
    const PatchDev P = patches[w.patch];
    if (!P.active) return;  // frozen patch (whole block)
    BoxPos bp = box_pos(P, w.a, Box{0, -1});
    double s = 0.0;
    if (bp.valid) {
        const int g = prm.ghost;
        long long x = sidx(P, bp.i + g, bp.j + g, bp.k + g);
        const R* q = pool + P.base + (long long)(cur ? F_ST1 : F_ST0) * P.vol;
        double u[8];
#pragma unroll
        for (int c = 0; c < 8; c++) u[c] = (double)q[(long long)c * P.vol + x];
        s = signal_speed(u, prm);
    }
    block_max_atomic(s, smax_bits);
}

__device__ __forceinline__ void write_step_const(StepConst* sc, double dt, const DevParams& p) {
    sc->dt = dt;
    sc->hdt = 0.5 * dt;
    sc->fdt = (float)dt;
    sc->fhdt = (float)(0.5 * dt);
    for (int d = 0; d < 3; d++) {
        sc->lam[d] = dt / p.dx[d];
        sc->il[d] = 0.5 * p.dx[d] / dt;
        sc->flam[d] = (float)sc->lam[d];
        sc->fil[d] = (float)sc->il[d];
    }
}

// smax_bits[0]: the maximum of the current state (folded by the update that
// produced it, or reduced explicitly); smax_bits[1]: that of the state one
// step earlier (0 right after an explicit reduction: nothing to lag behind).
// With dt_lag the step takes the earlier one (Sect. 4.1.1).
__global__ void dt_finalize_kernel(unsigned long long* smax_bits, StepConst* sc, DevParams p) {
    const unsigned long long cur = smax_bits[0], prev = smax_bits[1];
    const unsigned long long use = (p.dt_lag && prev != 0ULL) ? prev : cur;
    write_step_const(sc, p.cfl / __longlong_as_double((long long)use), p);
    smax_bits[1] = cur;
    smax_bits[0] = 0ULL;
}

__global__ void set_dt_kernel(StepConst* sc, double dt, DevParams p) { write_step_const(sc, dt, p); }

// clears both signal-speed slots before an explicit reduction
__global__ void zero_u64_kernel(unsigned long long* p) {
    p[0] = 0ULL;
    p[1] = 0ULL;
}

// ---------------------------------------------------------------------------
// Steps 3 and 9: upwinded edge EMFs from face fluxes and E^r.  For the edge of
// component c at the lower corner of the (a, b) = (c+1, c+2) plane, each of
// the four adjacent face values (-flux_a[B_b] on a-faces, +flux_b[B_a] on
// b-faces) is extrapolated half a zone to the edge with the face-to-centre
// difference on the upwind side (by the sign of the mass flux across the
// face carrying it; the average of both sides when it is exactly zero); the
// edge value is the mean of the four.
// ---------------------------------------------------------------------------

template <typename R>
__device__ __forceinline__ R upwind_pick(R f, R dl, R dr) {
    return f > R(0) ? dl : (f < R(0) ? dr : R(0.5) * (dl + dr));
}

// Upwinded edge value from preloaded face data: Ea_0, Ea_b the
// a-face values -flux_a[B_b] at the zone and one back along b; Eb_0, Eb_a the
// b-face values +flux_b[B_a] at the zone and one back along a; m* the mass
// fluxes across the same faces; e* the E^r of the four zones.
template <typename R>
__device__ __forceinline__ R edge_combine(R Ea_0, R Ea_b, R Eb_0, R Eb_a, R ma_0, R ma_b, R mb_0, R mb_a, R e0, R ea,
                                          R eb, R eab) {
    R d1 = upwind_pick(ma_0, ea - Eb_a, e0 - Eb_0);
    R d2 = upwind_pick(ma_b, Eb_a - eab, Eb_0 - eb);
    R d3 = upwind_pick(mb_0, eb - Ea_b, e0 - Ea_0);
    R d4 = upwind_pick(mb_a, Ea_b - eab, Ea_0 - ea);
    return R(0.25) * ((Ea_0 - d1) + (Ea_b + d2) + (Eb_0 - d3) + (Eb_a + d4));
}

// Column tiles of the marching kernels, ty <= 32.  Steps 3-4: tx <= 40 and
// tx ty <= 256 zones per plane, LDS edge planes (tx+1)(ty+1) <= 297 long.
// Steps 8-11: tx ty <= Z <= upd_tile_zones_max (the block size: 256 or 512),
// tx <= 48, the E^r planes (tx+2)(ty+2) <= upd_er_plane and the edge planes
// (tx+1)(ty+1) <= upd_ed_plane long (the tile planner caps ty for these),
// and the ring 2 (tx+2) + 2 ty <= Z.
constexpr int TILE_THREADS = 256;
constexpr int CTH_EDMAX = 297;
template <typename R>
struct UpdTile {
    static constexpr int threads = upd_tile_zones_max((int)sizeof(R));
    static constexpr int er = upd_er_plane((int)sizeof(R));
    static constexpr int ed = upd_ed_plane((int)sizeof(R));
};
constexpr int TILE_BIAS = 16;  // tile origins are stored biased (they may be negative)

// q = r / m for r, m >= 1 with r m < 65536, from a 16-bit reciprocal
__device__ __forceinline__ int small_div(int r, int recip) { return (r * recip) >> 16; }

// ---------------------------------------------------------------------------
// Steps 3-4 fused.  A block owns a column tile of the in-plane box
// [-2, n+2]^2 and marches over the planes z in [-2, n+2].  Iteration k forms
//   phase 1  the Step-3 edge EMFs of plane k+1 (Step-1 fluxes, E^r of Step 2)
//            into LDS, three planes deep, so one barrier a plane suffices,
//   phase 2  b^{n+1/2} = b^n - (dt/2) curl E (Step 4, Stokes form) on the
//            faces of plane k that the corrector reads: b_d with z_d in
//            [-2, n+2] and the transverse coordinates in [-1, n].
// The plane-below fluxes and E^r of the E_x and E_y edges are carried in
// registers, so each datum is read once.  An edge is needed only where its
// own coordinate is in [-1, n] and the others in [-2, n+2]; those outside
// are formed (from in-bounds ghost memory) but never read.
// ---------------------------------------------------------------------------

template <typename R>
__global__ void __launch_bounds__(TILE_THREADS) ct_half_kernel(R* __restrict__ pool, const PatchDev* __restrict__ patches,
                                                               const WorkItem* __restrict__ work, Coef<R> cf, int ghost,
                                                               int cur, const StepConst* __restrict__ sc) {
    __shared__ R s_ed[3 * 3 * CTH_EDMAX];  // [plane mod 3][component][j (tx+1) + i]
    const WorkItem w = work[blockIdx.x];
    if (w.patch < 0) return;  // padding item (whole block)
    const PatchDev P = patches[w.patch];
    if (!P.active) return;  // frozen patch (whole block, before any barrier)
    const int i0 = (w.a & 0xffff) - TILE_BIAS, j0 = (w.a >> 16) - TILE_BIAS;
    const int tx = w.b & 0xffff, ty = w.b >> 16;
    const int k0 = (w.c & 0xffff) - TILE_BIAS, k1 = (w.c >> 16) - TILE_BIAS;
    constexpr unsigned ES = sizeof(R);
    const int g = ghost;
    const unsigned VB = (unsigned)P.vol * ES;
    const unsigned s0 = ES, s1 = (unsigned)P.N[0] * ES, s2 = (unsigned)(P.N[0] * P.N[1]) * ES;
    const __amdgpu_buffer_rsrc_t rs = patch_rsrc(pool + P.base, (unsigned)F_STATE * VB);     // state
    const __amdgpu_buffer_rsrc_t rw = patch_rsrc(pool + P.sbase, (unsigned)F_SCRATCH * VB);  // step intermediates
    const unsigned bs = (unsigned)((cur ? F_ST1 : F_ST0) + 8) * VB;
    const unsigned FX = (unsigned)F_FL1 * VB, FY = FX + 7 * VB, FZ = FY + 7 * VB, ER = (unsigned)F_ER * VB;
    const R tau = sc_hdt(*sc, R(0));
    const R ix = cf.idx[0], iy = cf.idx[1], iz = cf.idx[2];
    const R z0 = R(0);
    const int t = threadIdx.x;
    const int TXE = tx + 1;
    auto zoff = [&](int i, int j, int k) -> unsigned {
        return (unsigned)sidx(P, i0 + i + g, j0 + j + g, k + g) * ES;
    };
    auto ld = [&](unsigned voff, unsigned soff) -> R { return bload(z0, rw, voff, soff); };

    const bool owner = t < tx * ty;
    const int zj = owner ? small_div(t, 65536 / tx + 1) : 0, zi = owner ? t - zj * tx : 0;
    const bool extra = t <= tx + ty;  // edges on the column i = tx, then on the row j = ty
    const int xi = t <= ty ? tx : t - ty - 1, xj = t <= ty ? t : ty;
    const int xmask = (xi < tx ? 1 : 0) | (xj < ty ? 2 : 0) | 4;

    // Step 3 at tile-local edge position (i, j) of plane p, components in mask.
    // cx: m_y, flux_y[B_z], E^r_x at (i, j) and E^r_x at (i, j-1) of plane p-1;
    // cy: m_x, flux_x[B_z], E^r_y at (i, j) and E^r_y at (i-1, j) of plane p-1
    // (carried, loaded when fresh); replaced by those of plane p.
    auto ed_item = [&](int i, int j, int p, int mask, R(&cx)[4], R(&cy)[4], bool fresh) {
        const unsigned xo = zoff(i, j, p);
        R* dst = s_ed + ((p + 3) % 3) * 3 * CTH_EDMAX + j * TXE + i;
        if (mask & 1) {  // E_x: a = y, b = z
            if (fresh) {
                cx[0] = ld(xo - s2, FY), cx[1] = ld(xo - s2, FY + 5 * VB);
                cx[2] = ld(xo - s2, ER), cx[3] = ld(xo - s2 - s1, ER);
            }
            const R ma = ld(xo, FY), fa5 = ld(xo, FY + 5 * VB);
            const R mb = ld(xo, FZ), fb6 = ld(xo, FZ + 6 * VB), mba = ld(xo - s1, FZ), fb6a = ld(xo - s1, FZ + 6 * VB);
            const R e0 = ld(xo, ER), ea = ld(xo - s1, ER);
            dst[0] = edge_combine(-fa5, -cx[1], fb6, fb6a, ma, cx[0], mb, mba, e0, ea, cx[2], cx[3]);
            cx[0] = ma, cx[1] = fa5, cx[2] = e0, cx[3] = ea;
        }
        if (mask & 2) {  // E_y: a = z, b = x
            if (fresh) {
                cy[0] = ld(xo - s2, FX), cy[1] = ld(xo - s2, FX + 6 * VB);
                cy[2] = ld(xo - s2, ER + VB), cy[3] = ld(xo - s2 - s0, ER + VB);
            }
            const R ma = ld(xo, FZ), fa5 = ld(xo, FZ + 5 * VB), mab = ld(xo - s0, FZ), fa5b = ld(xo - s0, FZ + 5 * VB);
            const R mb = ld(xo, FX), fb6 = ld(xo, FX + 6 * VB);
            const R e0 = ld(xo, ER + VB), eb = ld(xo - s0, ER + VB);
            dst[CTH_EDMAX] = edge_combine(-fa5, -fa5b, fb6, cy[1], ma, mab, mb, cy[0], e0, cy[2], eb, cy[3]);
            cy[0] = mb, cy[1] = fb6, cy[2] = e0, cy[3] = eb;
        }
        if (mask & 4) {  // E_z: a = x, b = y
            const R ma = ld(xo, FX), fa5 = ld(xo, FX + 5 * VB), mab = ld(xo - s1, FX), fa5b = ld(xo - s1, FX + 5 * VB);
            const R mb = ld(xo, FY), fb6 = ld(xo, FY + 6 * VB), mba = ld(xo - s0, FY), fb6a = ld(xo - s0, FY + 6 * VB);
            const unsigned ez = ER + 2 * VB;
            dst[2 * CTH_EDMAX] = edge_combine(-fa5, -fa5b, fb6, fb6a, ma, mab, mb, mba, ld(xo, ez), ld(xo - s0, ez),
                                              ld(xo - s1, ez), ld(xo - s0 - s1, ez));
        }
    };

    R cx_o[4], cy_o[4], cx_x[4], cy_x[4];
    const int gi = i0 + zi, gj = j0 + zj;
    const bool ix_in = gi >= -1 && gi <= P.n[0], jy_in = gj >= -1 && gj <= P.n[1];
    const int e = zj * TXE + zi;

    if (owner) ed_item(zi, zj, k0, 7, cx_o, cy_o, true);
    if (extra) ed_item(xi, xj, k0, xmask, cx_x, cy_x, true);
    for (int k = k0; k < k1; k++) {
        if (owner) ed_item(zi, zj, k + 1, 7, cx_o, cy_o, false);
        if (extra) ed_item(xi, xj, k + 1, xmask, cx_x, cy_x, false);
        __syncthreads();
        if (owner) {
            const bool kz_in = k >= -1 && k <= P.n[2];
            const unsigned xo = zoff(zi, zj, k);
            const R* ex0 = s_ed + ((k + 3) % 3) * 3 * CTH_EDMAX;  // E_x, plane k
            const R* ey0 = ex0 + CTH_EDMAX;
            const R* ez0 = ex0 + 2 * CTH_EDMAX;
            const R* ex1 = s_ed + ((k + 4) % 3) * 3 * CTH_EDMAX;  // E_x, plane k+1
            const R* ey1 = ex1 + CTH_EDMAX;
            if (jy_in && kz_in) {
                R curl = (ez0[e + TXE] - ez0[e]) * iy - (ey1[e] - ey0[e]) * iz;
                bstore(bload(z0, rs, xo, bs) - tau * curl, rw, xo, (unsigned)F_BH * VB);
            }
            if (ix_in && kz_in) {
                R curl = (ex1[e] - ex0[e]) * iz - (ez0[e + 1] - ez0[e]) * ix;
                bstore(bload(z0, rs, xo, bs + VB) - tau * curl, rw, xo, (unsigned)(F_BH + 1) * VB);
            }
            if (ix_in && jy_in) {
                R curl = (ey0[e + 1] - ey0[e]) * ix - (ex0[e + TXE] - ex0[e]) * iy;
                bstore(bload(z0, rs, xo, bs + 2 * VB) - tau * curl, rw, xo, (unsigned)(F_BH + 2) * VB);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Steps 8-11 fused.  A block owns a column tile of zones [i0, i0+tx) x
// [j0, j0+ty) (tx, ty <= 32, tx ty <= its block size) over the planes [k0, k1) and
// marches along z.  Iteration k forms
//   phase 1  E^r on plane k+1 over the tile and a one-zone ring (Step 8:
//            velocity of the unsplit half update of q^n with the Step-6/7
//            fluxes, zone field from the face average of b^{n+1/2}),
//   phase 2  the Step-9 edge EMFs of plane k+1 (the Step-3 upwinded average
//            with the fluxes of Steps 6/7),
//   phase 3  the zones of plane k: conservative update (Step 10), CT update
//            of their faces (Step 11), zone field from the face average,
//            FP64 floors, and the FP64 signal speed folded into smax.
// E^r and the edges live in LDS, two planes each.  Every value that a later
// plane needs again is carried in registers (z-face fluxes and fields, the
// plane-below fluxes of the E_x and E_y edges, the divergence of the own
// zone formed in phase 1), so each datum is read from memory once per step
// and the L2 only serves reuse within a plane.  Nothing of Steps 8-9 goes to
// HBM unless keep_edges asks for the Step-9 edges (debugging).  The new state
// of the first and last g zones of each interior row is also written into the
// x-ghosts of the x-neighbours, so the next ghost exchange needs only its y
// and z passes.
// ---------------------------------------------------------------------------

// One tile of Steps 8-11 (all threads of the block); returns the block's
// part of the signal-speed maximum of the new state (per thread).
template <typename R>
__device__ __forceinline__ double update_tile(const WorkItem w, R* __restrict__ pool,
                                              const PatchDev* __restrict__ patches, const DevParams& prm,
                                              const Coef<R>& cf, int cur, const StepConst* __restrict__ sc,
                                              unsigned long long* __restrict__ nfloor, int keep_edges,
                                              R* __restrict__ s_er, R* __restrict__ s_ed) {
    constexpr int UPD_ERMAX = UpdTile<R>::er, UPD_EDMAX = UpdTile<R>::ed;
    if (w.patch < 0) return 0.0;  // padding item (whole block)
    const PatchDev P = patches[w.patch];
    if (!P.active) return 0.0;  // frozen patch (whole block, before any barrier)
    const int i0 = (w.a & 0xffff) - TILE_BIAS, j0 = (w.a >> 16) - TILE_BIAS;
    const int tx = w.b & 0xffff, ty = w.b >> 16;
    const int k0 = (w.c & 0xffff) - TILE_BIAS, k1 = (w.c >> 16) - TILE_BIAS;
    constexpr unsigned ES = sizeof(R);
    const int g = prm.ghost;
    const unsigned VB = (unsigned)P.vol * ES;
    const unsigned s0 = ES, s1 = (unsigned)P.N[0] * ES, s2 = (unsigned)(P.N[0] * P.N[1]) * ES;
    const __amdgpu_buffer_rsrc_t rs = patch_rsrc(pool + P.base, (unsigned)F_STATE * VB);     // state
    const __amdgpu_buffer_rsrc_t rw = patch_rsrc(pool + P.sbase, (unsigned)F_SCRATCH * VB);  // step intermediates
    const unsigned qs = (unsigned)(cur ? F_ST1 : F_ST0) * VB, bs = qs + 8 * VB;
    const unsigned qn = (unsigned)(cur ? F_ST0 : F_ST1) * VB, bn = qn + 8 * VB;
    const unsigned FX = (unsigned)F_FL2 * VB, FY = FX + 7 * VB, FZ = FY + 7 * VB, BH = (unsigned)F_BH * VB;
    const R hdt = sc_hdt(*sc, R(0)), dt = sc_dt(*sc, R(0));
    const R ix = cf.idx[0], iy = cf.idx[1], iz = cf.idx[2];
    const R z0 = R(0);
    const int t = threadIdx.x;
    const int TXP = tx + 2, TXE = tx + 1;
    auto zoff = [&](int i, int j, int k) -> unsigned {
        return (unsigned)sidx(P, i0 + i + g, j0 + j + g, k + g) * ES;
    };
    auto ld = [&](unsigned voff, unsigned soff) -> R { return bload(z0, rw, voff, soff); };
    auto lds = [&](unsigned voff, unsigned soff) -> R { return bload(z0, rs, voff, soff); };

    // own zone (every thread of a full tile), ring zone of E^r, extra edge position
    const bool owner = t < tx * ty;
    const int zj = owner ? small_div(t, 65536 / tx + 1) : 0, zi = owner ? t - zj * tx : 0;
    const int nring = 2 * TXP + 2 * ty;
    const bool ring = t < nring;
    int rx = 0, ry = 0;
    if (t < TXP) {
        rx = t - 1, ry = -1;
    } else if (t < 2 * TXP) {
        rx = t - TXP - 1, ry = ty;
    } else if (t < 2 * TXP + ty) {
        rx = -1, ry = t - 2 * TXP;
    } else {
        rx = tx, ry = t - 2 * TXP - ty;
    }
    const bool extra = t <= tx + ty;  // edges on the column i = tx, then on the row j = ty
    const int xi = t <= ty ? tx : t - ty - 1, xj = t <= ty ? t : ty;
    const int xmask = (xi < tx ? 1 : 0) | (xj < ty ? 2 : 0) | 4;

    // Step 8 at tile-local zone (ex, ey) of plane p.  fz, bz: flux_z rows 0-3 and
    // b^{n+1/2}_z on the lower z-face (carried from plane p-1, loaded when
    // fresh); replaced by those of the upper face.  uf, if given, receives
    // q - dt div F of rows 0-3 for the final update of the zone; r0, if
    // given, the rho rows of flux_x, flux_y and flux_z on the zone's lower
    // faces, which the zone's edges of Step 9 use again.
    auto er_item = [&](int ex, int ey, int p, R(&fz)[4], R& bz, bool fresh, R* uf, R* r0) {
        const unsigned xo = zoff(ex, ey, p);
        R u[4];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const unsigned cf0 = FX + c * VB, cf1 = FY + c * VB, cf2 = FZ + c * VB;
            if (fresh) fz[c] = ld(xo, cf2);
            const R fzn = ld(xo + s2, cf2);
            const R fx = ld(xo, cf0), fy = ld(xo, cf1);
            if (c == 0 && r0) r0[0] = fx, r0[1] = fy, r0[2] = fz[0];
            R div = R(0);
            div += (ld(xo + s0, cf0) - fx) * ix;
            div += (ld(xo + s1, cf1) - fy) * iy;
            div += (fzn - fz[c]) * iz;
            const R q = lds(xo, qs + c * VB);
            u[c] = q - hdt * div;
            if (uf) uf[c] = q - dt * div;
            fz[c] = fzn;
        }
        if (fresh) bz = ld(xo, BH + 2 * VB);
        const R bzn = ld(xo + s2, BH + 2 * VB);
        R B0 = R(0.5) * (ld(xo, BH) + ld(xo + s0, BH));
        R B1 = R(0.5) * (ld(xo, BH + VB) + ld(xo + s1, BH + VB));
        R B2 = R(0.5) * (bz + bzn);
        bz = bzn;
        R ir = frcp(u[0]);
        R vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
        R* dst = s_er + (p & 1) * 3 * UPD_ERMAX + (ey + 1) * TXP + (ex + 1);
        dst[0] = vz * B1 - vy * B2;
        dst[UPD_ERMAX] = vx * B2 - vz * B0;
        dst[2 * UPD_ERMAX] = vy * B0 - vx * B1;
    };

    // Step 9 at tile-local edge position (i, j) of plane p, components in mask
    // (bit c).  cx: flux_y rows 0 and 5, cy: flux_x rows 0 and 6, both at (i, j)
    // of plane p-1 (carried, loaded when fresh); replaced by those of plane p.
    auto ed_item = [&](int i, int j, int p, int mask, R(&cx)[2], R(&cy)[2], bool fresh, const R* r0) {
        const unsigned xo = zoff(i, j, p);
        // the rho rows on the position's lower faces (from Step 8 when given)
        const R fx0 = r0 ? r0[0] : ld(xo, FX), fy0 = r0 ? r0[1] : ld(xo, FY), fz0 = r0 ? r0[2] : ld(xo, FZ);
        const int ri = (j + 1) * TXP + (i + 1), e = j * TXE + i;
        const R* ec = s_er + (p & 1) * 3 * UPD_ERMAX + ri;        // E^r of plane p at the edge's zone
        const R* ep = s_er + ((p - 1) & 1) * 3 * UPD_ERMAX + ri;  // plane p-1
        R* dst = s_ed + (p & 1) * 3 * UPD_EDMAX + e;
        if (mask & 1) {  // E_x: a = y, b = z
            if (fresh) cx[0] = ld(xo - s2, FY), cx[1] = ld(xo - s2, FY + 5 * VB);
            const R ma = fy0, fa5 = ld(xo, FY + 5 * VB);
            const R mb = fz0, fb6 = ld(xo, FZ + 6 * VB), mba = ld(xo - s1, FZ), fb6a = ld(xo - s1, FZ + 6 * VB);
            const R E = edge_combine(-fa5, -cx[1], fb6, fb6a, ma, cx[0], mb, mba, ec[0], ec[-TXP], ep[0], ep[-TXP]);
            dst[0] = E;
            if (keep_edges) bstore(E, rw, xo, (unsigned)F_ED * VB);
            cx[0] = ma, cx[1] = fa5;
        }
        if (mask & 2) {  // E_y: a = z, b = x
            if (fresh) cy[0] = ld(xo - s2, FX), cy[1] = ld(xo - s2, FX + 6 * VB);
            const R ma = fz0, fa5 = ld(xo, FZ + 5 * VB), mab = ld(xo - s0, FZ), fa5b = ld(xo - s0, FZ + 5 * VB);
            const R mb = fx0, fb6 = ld(xo, FX + 6 * VB);
            const R* c1 = ec + UPD_ERMAX;
            const R* p1 = ep + UPD_ERMAX;
            const R E = edge_combine(-fa5, -fa5b, fb6, cy[1], ma, mab, mb, cy[0], c1[0], p1[0], c1[-1], p1[-1]);
            dst[UPD_EDMAX] = E;
            if (keep_edges) bstore(E, rw, xo, (unsigned)(F_ED + 1) * VB);
            cy[0] = mb, cy[1] = fb6;
        }
        if (mask & 4) {  // E_z: a = x, b = y
            const R ma = fx0, fa5 = ld(xo, FX + 5 * VB), mab = ld(xo - s1, FX), fa5b = ld(xo - s1, FX + 5 * VB);
            const R mb = fy0, fb6 = ld(xo, FY + 6 * VB), mba = ld(xo - s0, FY), fb6a = ld(xo - s0, FY + 6 * VB);
            const R* c2 = ec + 2 * UPD_ERMAX;
            const R E = edge_combine(-fa5, -fa5b, fb6, fb6a, ma, mab, mb, mba, c2[0], c2[-1], c2[-TXP], c2[-1 - TXP]);
            dst[2 * UPD_EDMAX] = E;
            if (keep_edges) bstore(E, rw, xo, (unsigned)(F_ED + 2) * VB);
        }
    };

    // carried registers: E^r items (own, ring), edge items (own, extra), final update
    R fz_o[4], fz_r[4], bz_o = R(0), bz_r = R(0);
    R cx_o[2], cy_o[2], cx_x[2], cy_x[2];
    R ufc[4], ufn[4];  // q - dt div F (rows 0-3) of the own zone on planes k and k+1
    R r0o[3];          // rho rows of the own zone's lower-face fluxes (Step 8 -> Step 9)
    R fz4 = R(0), bzc = R(0);  // flux_z row 4 and b^{n+1}_z on the lower face of plane k
    double sp = 0.0;

    // prologue: E^r of planes k0-1 and k0, edges of plane k0
    if (owner) er_item(zi, zj, k0 - 1, fz_o, bz_o, true, nullptr, nullptr);
    if (ring) er_item(rx, ry, k0 - 1, fz_r, bz_r, true, nullptr, nullptr);
    if (owner) er_item(zi, zj, k0, fz_o, bz_o, false, ufc, r0o);
    if (ring) er_item(rx, ry, k0, fz_r, bz_r, false, nullptr, nullptr);
    __syncthreads();
    if (owner) ed_item(zi, zj, k0, 7, cx_o, cy_o, true, r0o);
    if (extra) ed_item(xi, xj, k0, xmask, cx_x, cy_x, true, nullptr);
    __syncthreads();
    for (int k = k0; k < k1; k++) {
        if (owner) er_item(zi, zj, k + 1, fz_o, bz_o, false, ufn, r0o);
        if (ring) er_item(rx, ry, k + 1, fz_r, bz_r, false, nullptr, nullptr);
        __syncthreads();
        if (owner) ed_item(zi, zj, k + 1, 7, cx_o, cy_o, false, r0o);
        if (extra) ed_item(xi, xj, k + 1, xmask, cx_x, cy_x, false, nullptr);
        __syncthreads();
        if (owner) {
            const unsigned xo = zoff(zi, zj, k);
            R u[8];
#pragma unroll
            for (int c = 0; c < 4; c++) u[c] = ufc[c];
            // Step 10 on E (flux row 4)
            {
                if (k == k0) fz4 = ld(xo, FZ + 4 * VB);
                const R fz4n = ld(xo + s2, FZ + 4 * VB);
                R div = R(0);
                div += (ld(xo + s0, FX + 4 * VB) - ld(xo, FX + 4 * VB)) * ix;
                div += (ld(xo + s1, FY + 4 * VB) - ld(xo, FY + 4 * VB)) * iy;
                div += (fz4n - fz4) * iz;
                u[7] = lds(xo, qs + 7 * VB) - dt * div;
                fz4 = fz4n;
            }
            const R* ex0 = s_ed + (k & 1) * 3 * UPD_EDMAX;  // E_x, plane k
            const R* ey0 = ex0 + UPD_EDMAX;                  // E_y, plane k
            const R* ez0 = ex0 + 2 * UPD_EDMAX;              // E_z, plane k
            const R* ex1 = s_ed + ((k + 1) & 1) * 3 * UPD_EDMAX;  // E_x, plane k+1
            const R* ey1 = ex1 + UPD_EDMAX;                        // E_y, plane k+1
            const int e = zj * TXE + zi;
            // Step 11 on the two faces of the zone along each axis (the lower
            // z-face is the upper one of the plane below)
            R bxl = lds(xo, bs) - dt * ((ez0[e + TXE] - ez0[e]) * iy - (ey1[e] - ey0[e]) * iz);
            R bxr = lds(xo + s0, bs) - dt * ((ez0[e + 1 + TXE] - ez0[e + 1]) * iy - (ey1[e + 1] - ey0[e + 1]) * iz);
            R byl = lds(xo, bs + VB) - dt * ((ex1[e] - ex0[e]) * iz - (ez0[e + 1] - ez0[e]) * ix);
            R byr = lds(xo + s1, bs + VB) -
                    dt * ((ex1[e + TXE] - ex0[e + TXE]) * iz - (ez0[e + 1 + TXE] - ez0[e + TXE]) * ix);
            if (k == k0) bzc = lds(xo, bs + 2 * VB) - dt * ((ey0[e + 1] - ey0[e]) * ix - (ex0[e + TXE] - ex0[e]) * iy);
            R bzl = bzc;
            R bzr = lds(xo + s2, bs + 2 * VB) - dt * ((ey1[e + 1] - ey1[e]) * ix - (ex1[e + TXE] - ex1[e]) * iy);
            bzc = bzr;
            bstore(bxl, rs, xo, bn);
            bstore(byl, rs, xo, bn + VB);
            bstore(bzl, rs, xo, bn + 2 * VB);
            // shared right faces of the patch
            // (face n along x is the +x neighbour's face 0, which it writes
            // here itself: pushed, or pulled below when it is frozen)
            if (i0 + zi == P.n[0] - 1 && P.nb[1] < 0) bstore(bxr, rs, xo + s0, bn);
            if (j0 + zj == P.n[1] - 1) bstore(byr, rs, xo + s1, bn + VB);
            if (k == P.n[2] - 1) bstore(bzr, rs, xo + s2, bn + 2 * VB);
            u[4] = R(0.5) * (bxl + bxr);
            u[5] = R(0.5) * (byl + byr);
            u[6] = R(0.5) * (bzl + bzr);
            if (apply_floor(u, prm, cf)) atomicAdd(nfloor, 1ULL);
#pragma unroll
            for (int c = 0; c < 8; c++) bstore(u[c], rs, xo, qn + c * VB);
            // ghost exchange along x, pushed: the first and last g zones of an
            // interior row are the x-ghosts of the -x and +x neighbours (same
            // row and plane, face neighbours share the y-z extent); at a domain
            // boundary (no neighbour) the boundary zone fills the patch's own
            // x-ghosts by zero gradient, b_x from the boundary face
            const int gi = i0 + zi;
#pragma unroll
            for (int side = 0; side < 2; side++) {
                const bool mine = side == 0 ? gi < g : gi >= P.n[0] - g;
                if (!mine) continue;
                const int nbq = P.nb[side];
                if (nbq >= 0) {
                    const PatchDev Q = patches[nbq];
                    const int qi = side == 0 ? Q.n[0] + gi : gi - P.n[0];
                    const unsigned QB = (unsigned)Q.vol * ES;
                    const __amdgpu_buffer_rsrc_t rq = patch_rsrc(pool + Q.base, (unsigned)F_STATE * QB);
                    const unsigned yo = (unsigned)sidx(Q, qi + g, j0 + zj + g, k + g) * ES;
                    const unsigned qq = (unsigned)(cur ? F_ST0 : F_ST1) * QB;
#pragma unroll
                    for (int c = 0; c < 8; c++) bstore(u[c], rq, yo, qq + c * QB);
                    bstore(bxl, rq, yo, qq + 8 * QB);
                    bstore(byl, rq, yo, qq + 9 * QB);
                    bstore(bzl, rq, yo, qq + 10 * QB);
                    // the upper y and z faces of the last row / plane: the
                    // boundary faces a wall-ended axis owns (elsewhere the
                    // y/z exchange overwrites them)
                    if (j0 + zj == P.n[1] - 1) bstore(byr, rq, yo + (unsigned)Q.N[0] * ES, qq + 9 * QB);
                    if (k == P.n[2] - 1) bstore(bzr, rq, yo + (unsigned)(Q.N[0] * Q.N[1]) * ES, qq + 10 * QB);
                    if (!Q.active) {
                        // a frozen neighbour pushes nothing: pull its zone into
                        // this patch's own x-ghost (its state is the same in
                        // both copies); the mirror image of the push above
                        const int xs = side == 0 ? gi : gi + 2 * g;                    // own ghost, stored x
                        const int xq = side == 0 ? Q.n[0] + gi : gi - P.n[0] + 2 * g;  // Q's zone, stored x
                        const unsigned yq = (unsigned)sidx(Q, xq, j0 + zj + g, k + g) * ES;
                        const unsigned yp = (unsigned)sidx(P, xs, j0 + zj + g, k + g) * ES;
                        const unsigned qc = (unsigned)(cur ? F_ST1 : F_ST0) * QB;
#pragma unroll
                        for (int c = 0; c < 11; c++) bstore(bload(z0, rq, yq, qc + c * QB), rs, yp, qn + c * VB);
                        if (j0 + zj == P.n[1] - 1)
                            bstore(bload(z0, rq, yq + (unsigned)Q.N[0] * ES, qc + 9 * QB), rs, yp + s1, bn + VB);
                        if (k == P.n[2] - 1)
                            bstore(bload(z0, rq, yq + (unsigned)(Q.N[0] * Q.N[1]) * ES, qc + 10 * QB), rs, yp + s2,
                                   bn + 2 * VB);
                    }
                } else if (gi == (side == 0 ? 0 : P.n[0] - 1)) {
                    const R bxg = side == 0 ? bxl : bxr;  // the boundary face
                    for (int m = 1; m <= g; m++) {
                        const unsigned yo = side == 0 ? xo - (unsigned)m * s0 : xo + (unsigned)m * s0;
#pragma unroll
                        for (int c = 0; c < 8; c++) bstore(u[c], rs, yo, qn + c * VB);
                        bstore(byl, rs, yo, bn + VB);
                        bstore(bzl, rs, yo, bn + 2 * VB);
                        if (side == 0 || m >= 2) bstore(bxg, rs, yo, bn);  // face n itself is stored above
                        if (j0 + zj == P.n[1] - 1) bstore(byr, rs, yo + s1, bn + VB);
                        if (k == P.n[2] - 1) bstore(bzr, rs, yo + s2, bn + 2 * VB);
                    }
                }
            }
            double ud[8];
#pragma unroll
            for (int c = 0; c < 8; c++) ud[c] = (double)u[c];
            sp = fmax(sp, signal_speed(ud, prm));
#pragma unroll
            for (int c = 0; c < 4; c++) ufc[c] = ufn[c];
        }
    }
    return sp;
}

// QUEUE = false: block b takes item b of the list.  QUEUE = true: a
// persistent grid whose block b, on XCD b mod 8 (blocks go to the XCDs
// round-robin), takes the items of that XCD's queue in the list (positions
// 8 j + x, the order xcd_order gives) one after another from an atomic
// counter; the last block to finish sets the counters back to zero, so the
// launch needs no reset of its own (and none inside a captured graph).
template <typename R, bool QUEUE>
__global__ void __launch_bounds__(UpdTile<R>::threads) update_kernel(R* __restrict__ pool, const PatchDev* __restrict__ patches,
                                                              const WorkItem* __restrict__ work, int nitems,
                                                              unsigned int* __restrict__ queue, DevParams prm, Coef<R> cf,
                                                              int cur, const StepConst* __restrict__ sc,
                                                              unsigned long long* __restrict__ nfloor,
                                                              unsigned long long* __restrict__ smax_bits, int keep_edges) {
    constexpr int UPD_ERMAX = UpdTile<R>::er, UPD_EDMAX = UpdTile<R>::ed;
    __shared__ R s_er[2 * 3 * UPD_ERMAX];  // [plane & 1][component][(ey+1)(tx+2) + ex+1]
    __shared__ R s_ed[2 * 3 * UPD_EDMAX];  // [plane & 1][component][j (tx+1) + i]
    double sp = 0.0;
    if (!QUEUE) {
        sp = update_tile<R>(work[blockIdx.x], pool, patches, prm, cf, cur, sc, nfloor, keep_edges, s_er, s_ed);
    } else {
        __shared__ int s_item;
        const int x = (int)(blockIdx.x & 7u), nq = nitems / 8;
        for (;;) {
            if (threadIdx.x == 0) s_item = (int)atomicAdd(queue + x, 1u);
            __syncthreads();
            const int j = s_item;
            __syncthreads();  // every thread has read s_item (and left the last tile's LDS)
            if (j >= nq) break;
            sp = fmax(sp, update_tile<R>(work[8 * j + x], pool, patches, prm, cf, cur, sc, nfloor, keep_edges, s_er,
                                         s_ed));
        }
        __threadfence();
        if (threadIdx.x == 0 && atomicAdd(queue + 8, 1u) == gridDim.x - 1) {
            // the last block: every block has made its last take
            for (int q = 0; q < 9; q++) atomicExch(queue + q, 0u);
        }
    }
    block_max_atomic(sp, smax_bits);
}

// ---------------------------------------------------------------------------
// MHDTVD directional sweep (Appendix A; Step 1 when STAGE == 1, Steps 5-7
// when STAGE == 2).  A block holds W pencils of P zones along D; every thread
// owns one zone of one pencil and, after a barrier, the face on its left.
// The pencils of a patch are numbered fast-transverse-first and a block takes
// W consecutive ones, so no lanes idle on partial tiles.
//
//   phase A  zone state -> primitives (rho, v_par, v_t1, v_t2, B_t1, B_t2, P)
//            and the zone's physical flux terms in LDS
//            (STAGE 2 first builds the predictor state q^{n+1/2}_D from q^n,
//             the transverse Step-1 fluxes and the div-B source, with FP64
//             floors; STAGE 1 along x also writes the Step-2 reference EMF)
//   phase B  face s (zones s-1, s): Roe average, eigen-speeds, characteristic
//            jumps alpha_k, nu_k, g-tilde_k -> LDS
//   phase C  faces 2 .. P-2: limiter g of both zones, gamma_k, beta_k, the
//            correction sum_k beta_k R_k, modified flux (7 rows) -> HBM
//
// The characteristic algebra is done in the primitive-like variables
// (rho, v, B_t, P) in which the Roe matrix is the textbook primitive matrix:
// alpha_k = L_k . (d rho, d v, d B_t, dP + X d rho) and the correction
// sum_k beta_k R_k is assembled there and mapped to conserved variables once.
// ---------------------------------------------------------------------------

// One LDS record per thread: 7 values padded to 8 so a record is read with
// vector loads (two 16-byte reads in FP32).
template <typename R>
struct alignas(8 * sizeof(R)) Rec8 {
    R v[8];
};

template <typename R>
struct FaceEig {
    R rho, sq, vx, vy, vz, b1, b2, X;
    R a2, a, cf, cs, alf, als, by, bz, s;
};

// Protection trigger of a face (protection floors set): the Roe sound speed
// squared before its floor clamp is not positive, or one of the six states
// inside the Roe fan, u_L + sum_{k<m} alpha_k R_k (m = 1..6), has a density
// below rho_prot or a pressure below p_prot.  The fan is walked in the
// primitive-like variables (rho, v, B_t, P'), each wave's increment mapped to
// conserved variables at the Roe state; u_L is the left rebuilt face state.
template <typename R>
__device__ __forceinline__ bool fan_below_floor(R rl, R vxl, R vyl, R vzl, R b1l, R b2l, R pl, R bf,
                                                const FaceEig<R>& e, R a2raw, const R alpha[7], const Coef<R>& cf) {
#pragma clang fp contract(on)
    if (a2raw <= R(0)) return true;
    R w0 = rl, w1 = rl * vxl, w2 = rl * vyl, w3 = rl * vzl, w5 = b1l, w6 = b2l;
    R w7 = pl * cf.igm1 + R(0.5) * rl * (vxl * vxl + vyl * vyl + vzl * vzl) + R(0.5) * (bf * bf + b1l * b1l + b2l * b2l);
    const R v2 = e.vx * e.vx + e.vy * e.vy + e.vz * e.vz;
    const R eh = R(0.5) * v2 + cf.gm2 * e.X * cf.igm1;
    const R sqa = e.sq * e.a, ra2 = e.rho * e.a2;
    bool low = false;
#pragma unroll
    for (int m = 0; m < 6; m++) {
        // primitive-like right eigenvector of wave m (ascending eigenvalue order)
        R dr, dvp, dv1, dv2, db1, db2, dp;
        const R sg = m < 3 ? R(-1) : R(1);
        if (m == 0) {  // fast, v - cf
            dr = e.rho * e.alf, dvp = sg * e.alf * e.cf, dv1 = -sg * e.als * e.cs * e.s * e.by,
            dv2 = -sg * e.als * e.cs * e.s * e.bz, db1 = sqa * e.als * e.by, db2 = sqa * e.als * e.bz, dp = ra2 * e.alf;
        } else if (m == 1 || m == 5) {  // Alfven
            dr = R(0), dvp = R(0), dv1 = -e.bz, dv2 = e.by, db1 = sg * e.s * e.sq * e.bz, db2 = -sg * e.s * e.sq * e.by,
            dp = R(0);
        } else if (m == 3) {  // entropy
            dr = R(1), dvp = R(0), dv1 = R(0), dv2 = R(0), db1 = R(0), db2 = R(0), dp = R(0);
        } else {  // slow, v -/+ cs
            dr = e.rho * e.als, dvp = sg * e.als * e.cs, dv1 = sg * e.alf * e.cf * e.s * e.by,
            dv2 = sg * e.alf * e.cf * e.s * e.bz, db1 = -sqa * e.alf * e.by, db2 = -sqa * e.alf * e.bz, dp = ra2 * e.als;
        }
        const R am = alpha[m];
        w0 += am * dr;
        w1 += am * (e.vx * dr + e.rho * dvp);
        w2 += am * (e.vy * dr + e.rho * dv1);
        w3 += am * (e.vz * dr + e.rho * dv2);
        w5 += am * db1;
        w6 += am * db2;
        w7 += am * (eh * dr + e.rho * (e.vx * dvp + e.vy * dv1 + e.vz * dv2) + e.b1 * db1 + e.b2 * db2 + dp * cf.igm1);
        const R pm = cf.gm1 * (w7 - R(0.5) * (w1 * w1 + w2 * w2 + w3 * w3) / w0 - R(0.5) * (bf * bf + w5 * w5 + w6 * w6));
        low |= (w0 < cf.rho_prot) || (pm < cf.p_prot);
    }
    return low;
}

// ---------------------------------------------------------------------------
// The three phases of a directional sweep as functions of values, shared by
// the two forms of the sweep (the LDS pencil kernel and the marching kernel)
// so that both compute every face with the same arithmetic.
// ---------------------------------------------------------------------------

// Phase A.  The zone state along the sweep frame of axis D (STAGE 2 first
// builds the predictor state q^{n+1/2}_D from q^n, the transverse Step-1
// fluxes and the div-B source, with FP64 floors) -> primitive record
// (rho, v_par, v_t1, v_t2, B_t1, B_t2, P clamped at p_floor, 1/sqrt(rho)).
// Split into the loads (zone_fetch) and the arithmetic (zone_record), so
// that the marching form can issue a zone's loads one zone ahead.
template <typename R, int STAGE>
struct ZoneRaw {
    R q[8];
    // STAGE 2: the transverse Step-1 flux rows at the zone and one zone up
    // along A1 (fa) and A2 (fb): rows 0-4, then B_D's rows (A1 row 6, A2 row
    // 5), then B_A1's (A2 row 6) and B_A2's (A1 row 5); the face field at
    // the zone's lower and upper faces along each axis
    R fa[STAGE == 2 ? 7 : 1][2], fb[STAGE == 2 ? 7 : 1][2], b[STAGE == 2 ? 3 : 1][2];
};

// rs: the patch's state, rw: its step intermediates (the Step-1 fluxes).
// STAGE 3: the corrector along D from the predictor records that the fused
// x/y corrector stored in the rows of D's corrector flux (q[0..6]: rho,
// v_D, v_A1, v_A2, B_A1, B_A2, P), each read once before its slot is
// overwritten by the flux of the same pencil.
template <typename R, int D, int STAGE>
__device__ __forceinline__ void zone_fetch(__amdgpu_buffer_rsrc_t rs, __amdgpu_buffer_rsrc_t rw, unsigned xo,
                                           const unsigned st[3], unsigned qs, unsigned VB, ZoneRaw<R, STAGE>& z) {
    constexpr int A1 = (D + 1) % 3, A2 = (D + 2) % 3;
    constexpr unsigned ES = sizeof(R);
    const R z0 = R(0);
    if (STAGE == 3) {
#pragma unroll
        for (int r = 0; r < 7; r++) z.q[r] = bload(z0, rw, xo, (unsigned)(F_FL2 + 7 * D + r) * VB);
        return;
    }
#pragma unroll
    for (int c = 0; c < 8; c++) z.q[c] = bload(z0, rs, xo, qs + c * VB);
    if (STAGE == 2) {
        const unsigned f1 = (unsigned)(F_FL1 + 7 * A1) * VB, f2 = (unsigned)(F_FL1 + 7 * A2) * VB;
        const unsigned s1 = st[A1] * ES, s2 = st[A2] * ES;
#pragma unroll
        for (int r = 0; r < 7; r++) {
            // rows 0-4, then A1's row 6 / A2's row 5 (B_D), then A1's row 5 / A2's row 6
            const int ra = r < 5 ? r : (r == 5 ? 6 : 5), rb = r < 5 ? r : (r == 5 ? 5 : 6);
            z.fa[r][0] = bload(z0, rw, xo, f1 + ra * VB);
            z.fa[r][1] = bload(z0, rw, xo, f1 + ra * VB + s1);
            z.fb[r][0] = bload(z0, rw, xo, f2 + rb * VB);
            z.fb[r][1] = bload(z0, rw, xo, f2 + rb * VB + s2);
        }
        const unsigned bs = qs + 8 * VB;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            z.b[a][0] = bload(z0, rs, xo, bs + a * VB);
            z.b[a][1] = bload(z0, rs, xo, bs + a * VB + st[a] * ES);
        }
    }
}

template <typename R, int D, int STAGE>
__device__ __forceinline__ Rec8<R> zone_record(const ZoneRaw<R, STAGE>& z, const Coef<R>& cf, const DevParams& prm,
                                               const StepConst& sc) {
#pragma clang fp contract(on)
    constexpr int A1 = (D + 1) % 3, A2 = (D + 2) % 3;
    if (STAGE == 3) {
        Rec8<R> rec;
#pragma unroll
        for (int r = 0; r < 7; r++) rec.v[r] = z.q[r];
        rec.v[7] = frsq(z.q[0]);
        return rec;
    }
    R u[8];
#pragma unroll
    for (int c = 0; c < 8; c++) u[c] = z.q[c];
    if (STAGE == 2) {
        // q^n values the div-B source needs (before the update below)
        const R q0 = u[0], q1 = u[1 + A1], q2 = u[1 + A2];
        const R B0[3] = {u[4], u[5], u[6]};
        const R hdt = sc_hdt(sc, R(0));
        const R i1 = cf.idx[A1], i2 = cf.idx[A2];
        // rho, m, E (rows 0..4 -> components 0,1,2,3,7)
#pragma unroll
        for (int r = 0; r < 5; r++) {
            const int c = r < 4 ? r : 7;
            R div = (z.fa[r][1] - z.fa[r][0]) * i1 + (z.fb[r][1] - z.fb[r][0]) * i2;
            u[c] -= hdt * div;
        }
        // B_D: flux_A1 row 6 (B_{A1+2}) and flux_A2 row 5 (B_{A2+1})
        {
            R div = (z.fa[5][1] - z.fa[5][0]) * i1 + (z.fb[5][1] - z.fb[5][0]) * i2;
            u[4 + D] -= hdt * div;
        }
        // B_A1 only from flux_A2 row 6; B_A2 only from flux_A1 row 5
        u[4 + A1] -= hdt * ((z.fb[6][1] - z.fb[6][0]) * i2);
        u[4 + A2] -= hdt * ((z.fa[6][1] - z.fa[6][0]) * i1);
        // div-B source (Gardiner & Stone 2008 form): momentum B dB_D/dx_D,
        // B_t v_t minmod(dB_D/dx_D, -dB_t'/dx_t'), energy B_t . S[B_t]
        R dB[3];
#pragma unroll
        for (int a = 0; a < 3; a++) dB[a] = (z.b[a][1] - z.b[a][0]) * cf.idx[a];
        R ir0 = frcp(q0);
        R v1 = q1 * ir0, v2 = q2 * ir0;
        R B1 = B0[A1], B2 = B0[A2];
        R sB1 = v1 * minmod2(dB[D], -dB[A2]);
        R sB2 = v2 * minmod2(dB[D], -dB[A1]);
#pragma unroll
        for (int c = 0; c < 3; c++) u[1 + c] += hdt * B0[c] * dB[D];
        u[4 + A1] += hdt * sB1;
        u[4 + A2] += hdt * sB2;
        u[7] += hdt * (B1 * sB1 + B2 * sB2);
        apply_floor(u, prm, cf);
    }
    R rho = u[0];
    // 1/sqrt(rho) once per zone: the faces form sqrt(rho), 1/rho and the
    // Roe density's reciprocal from it
    R rsq = frsq(rho);
    R ir = rsq * rsq;
    R vpar = u[1 + D] * ir, vt1 = u[1 + A1] * ir, vt2 = u[1 + A2] * ir;
    R b2 = u[4] * u[4] + u[5] * u[5] + u[6] * u[6];
    R pr = cf.gm1 * (u[7] - R(0.5) * rho * (vpar * vpar + vt1 * vt1 + vt2 * vt2) - R(0.5) * b2);
    if (pr < cf.p_floor) pr = cf.p_floor;
    Rec8<R> rec;
    rec.v[0] = rho;
    rec.v[1] = vpar;
    rec.v[2] = vt1;
    rec.v[3] = vt2;
    rec.v[4] = u[4 + A1];
    rec.v[5] = u[4 + A2];
    rec.v[6] = pr;
    rec.v[7] = rsq;
    return rec;
}

template <typename R, int D, int STAGE>
__device__ __forceinline__ Rec8<R> zone_phase(__amdgpu_buffer_rsrc_t rs, __amdgpu_buffer_rsrc_t rw, unsigned xo,
                                              const unsigned st[3], unsigned qs, unsigned VB, const Coef<R>& cf,
                                              const DevParams& prm, const StepConst& sc) {
    ZoneRaw<R, STAGE> z;
    zone_fetch<R, D, STAGE>(rs, rw, xo, st, qs, VB, z);
    return zone_record<R, D, STAGE>(z, cf, prm, sc);
}

// Phase B.  Face between zones L and Rr with B_par = bf: Roe average,
// eigen-speeds, characteristic jumps alpha_k, nu_k and g-tilde_k; with
// protection floors set, the trigger (a protected face then contributes no
// g-tilde).
template <typename R, bool PROT>
__device__ __forceinline__ void face_phase(const Rec8<R>& L, const Rec8<R>& Rr, R bf, R lam, const Coef<R>& cf,
                                           FaceEig<R>& e, R alpha[7], R nu[7], Rec8<R>& gr, bool& prot) {
#pragma clang fp contract(on)
    R rl = L.v[0], vxl = L.v[1], vyl = L.v[2], vzl = L.v[3], b1l = L.v[4], b2l = L.v[5], pl = L.v[6];
    R rr = Rr.v[0], vxr = Rr.v[1], vyr = Rr.v[2], vzr = Rr.v[3], b1r = Rr.v[4], b2r = Rr.v[5], prr = Rr.v[6];

    R bf2 = bf * bf;
    const R rsl = L.v[7], rsr = Rr.v[7];  // 1/sqrt(rho) of the two zones
    R hl = (cf.ggm * pl + R(0.5) * rl * (vxl * vxl + vyl * vyl + vzl * vzl) + bf2 + b1l * b1l + b2l * b2l) * (rsl * rsl);
    R hr = (cf.ggm * prr + R(0.5) * rr * (vxr * vxr + vyr * vyr + vzr * vzr) + bf2 + b1r * b1r + b2r * b2r) * (rsr * rsr);
    R sl = rl * rsl, sr = rr * rsr;
    R isum = frcp(sl + sr);
    e.rho = sl * sr;
    e.vx = (sl * vxl + sr * vxr) * isum;
    e.vy = (sl * vyl + sr * vyr) * isum;
    e.vz = (sl * vzl + sr * vzr) * isum;
    R h = (sl * hl + sr * hr) * isum;
    e.b1 = (sr * b1l + sl * b1r) * isum;
    e.b2 = (sr * b2l + sl * b2r) * isum;
    R db1 = b1r - b1l, db2 = b2r - b2l;
    e.X = (db1 * db1 + db2 * db2) * R(0.5) * isum * isum;
    R v2 = e.vx * e.vx + e.vy * e.vy + e.vz * e.vz;
    R bt2 = e.b1 * e.b1 + e.b2 * e.b2;
    R irho = rsl * rsr;  // 1 / (sqrt(rho_L) sqrt(rho_R))
    R a2 = cf.gm1 * (h - R(0.5) * v2 - (bf2 + bt2) * irho) - cf.gm2 * e.X;
    const R a2raw = a2;
    R a2min = cf.gam * cf.p_floor * irho;
    if (a2 < a2min) a2 = a2min;
    R ca2 = bf2 * irho, bp2 = bt2 * irho;
    R dpr = a2 - ca2 - bp2;
    R dd = fsqrt(dpr * dpr + R(4) * a2 * bp2);
    R cf2 = R(0.5) * (a2 + ca2 + bp2 + dd);
    const R rcf = frsq(cf2);  // 1/cf
    R cs2 = a2 * ca2 * (rcf * rcf);
    if (dd <= cf.tol * (a2 + ca2 + bp2)) {
        e.alf = R(1);
        e.als = R(0);
    } else {
        R af2, as2;
        if (dpr >= R(0)) {
            af2 = R(0.5) * (dd + dpr);
            as2 = a2 * bp2 * frcp(af2);
        } else {
            as2 = R(0.5) * (dd - dpr);
            af2 = a2 * bp2 * frcp(as2);
        }
        R idd = frcp(dd);
        e.alf = fsqrt(af2 * idd);
        e.als = fsqrt(as2 * idd);
    }
    if (bt2 <= cf.tol2 * (bf2 + bt2)) {
        e.by = R(0.70710678118654752440);
        e.bz = R(0.70710678118654752440);
    } else {
        R ib = frsq(bt2);
        e.by = e.b1 * ib;
        e.bz = e.b2 * ib;
    }
    e.s = bf >= R(0) ? R(1) : R(-1);
    const R isq = frsq(e.rho), ra = frsq(a2);  // 1/sqrt(rho), 1/a
    e.sq = e.rho * isq;
    e.a2 = a2;
    e.a = a2 * ra;
    e.cf = cf2 * rcf;
    e.cs = fsqrt(cs2);
    R ca = fsqrt(ca2);

    // characteristic jumps: alpha_k = L_k . (d rho, d v, d B_t, dP + X d rho)
    R drho = rr - rl;
    R dvx = vxr - vxl, dvy = vyr - vyl, dvz = vzr - vzl;
    R dp = (prr - pl) + e.X * drho;
    R dvpar = e.by * dvy + e.bz * dvz, dvper = -e.bz * dvy + e.by * dvz;
    R dbpar = e.by * db1 + e.bz * db2, dbper = -e.bz * db1 + e.by * db2;
    R ia2 = ra * ra;
    R i2a2 = R(0.5) * ia2;
    R ipa = R(0.5) * isq * ra;
    R pterm = dp * irho * i2a2;
    R Ef = e.alf * pterm + e.als * dbpar * ipa;
    R Of = (e.alf * e.cf * dvx - e.als * e.cs * e.s * dvpar) * i2a2;
    R Es = e.als * pterm - e.alf * dbpar * ipa;
    R Os = (e.als * e.cs * dvx + e.alf * e.cf * e.s * dvpar) * i2a2;
    R Ea = R(0.5) * dvper;
    R Oa = -R(0.5) * e.s * dbper * isq;
    alpha[0] = Ef - Of;
    alpha[6] = Ef + Of;
    alpha[2] = Es - Os;
    alpha[4] = Es + Os;
    alpha[1] = Ea - Oa;
    alpha[5] = Ea + Oa;
    alpha[3] = drho - dp * ia2;
    R ev[7] = {e.vx - e.cf, e.vx - ca, e.vx - e.cs, e.vx, e.vx + e.cs, e.vx + ca, e.vx + e.cf};
#pragma unroll
    for (int k = 0; k < 7; k++) {
        nu[k] = lam * ev[k];
        gr.v[k] = R(0.5) * (qvisc(nu[k], cf.eps[k], cf.q4e[k]) - nu[k] * nu[k]) * alpha[k];
    }
    gr.v[7] = R(0);
    prot = false;
    if (PROT) {
        // protected face: HLL flux, no g-tilde for the limiters
        prot = fan_below_floor(rl, vxl, vyl, vzl, b1l, b2l, pl, bf, e, a2raw, alpha, cf);
        if (prot)
#pragma unroll
            for (int k = 0; k < 7; k++) gr.v[k] = R(0);
    }
}

// Physical fluxes of the two rebuilt face states (B_par = bf), the frame's 7
// rows (rho, m_par, m_t1, m_t2, E, B_t1, B_t2).
template <typename R>
__device__ __forceinline__ void face_fluxes(const Rec8<R>& Z, R bf, const Coef<R>& cf, R F[7]) {
#pragma clang fp contract(on)
    R r = Z.v[0], vx = Z.v[1], vy = Z.v[2], vz = Z.v[3], b1 = Z.v[4], b2 = Z.v[5], pr = Z.v[6];
    R bb = bf * bf + b1 * b1 + b2 * b2;
    R pt = pr + R(0.5) * bb;
    R ept = cf.ggm * pr + R(0.5) * r * (vx * vx + vy * vy + vz * vz) + bb;  // E + P*
    R mx = r * vx;
    F[0] = mx;
    F[1] = mx * vx + pt - bf * bf;
    F[2] = mx * vy - bf * b1;
    F[3] = mx * vz - bf * b2;
    F[4] = ept * vx - bf * (bf * vx + b1 * vy + b2 * vz);
    F[5] = b1 * vx - bf * vy;
    F[6] = b2 * vx - bf * vz;
}

// The flux part that needs no limiter: half the sum of the two states'
// physical fluxes, or for a protected face the whole HLL flux (Einfeldt
// bounds): (b+ F_L - b- F_R + b+ b- (u_R - u_L)) / (b+ - b-).
template <typename R, bool PROT>
__device__ __forceinline__ void face_central(const Rec8<R>& ZL, const Rec8<R>& ZR, R bf, const FaceEig<R>& e, bool prot,
                                             const Coef<R>& cf, R cav[7]) {
#pragma clang fp contract(on)
    R F[2][7];
    face_fluxes(ZL, bf, cf, F[0]);
    face_fluxes(ZR, bf, cf, F[1]);
#pragma unroll
    for (int r = 0; r < 7; r++) cav[r] = R(0.5) * (F[0][r] + F[1][r]);
    if (PROT && prot) {
        R U[2][7], vfs[2];
#pragma unroll
        for (int side = 0; side < 2; side++) {
            const Rec8<R>& Z = side ? ZR : ZL;
            R r = Z.v[0], vx = Z.v[1], vy = Z.v[2], vz = Z.v[3], b1 = Z.v[4], b2 = Z.v[5], pr = Z.v[6];
            U[side][0] = r;
            U[side][1] = r * vx;
            U[side][2] = r * vy;
            U[side][3] = r * vz;
            U[side][4] = pr * cf.igm1 + R(0.5) * r * (vx * vx + vy * vy + vz * vz) + R(0.5) * (bf * bf + b1 * b1 + b2 * b2);
            U[side][5] = b1;
            U[side][6] = b2;
            // fast speed of the rebuilt state along the sweep
            R ir = frcp(r);
            R fa2 = cf.gam * pr * ir, fca2 = bf * bf * ir, fbp2 = (b1 * b1 + b2 * b2) * ir;
            R fdp = fa2 - fca2 - fbp2;
            R fcf = fsqrt(R(0.5) * (fa2 + fca2 + fbp2 + fsqrt(fdp * fdp + R(4) * fa2 * fbp2)));
            vfs[side] = side ? vx + fcf : vx - fcf;
        }
        const R bp = fmax(fmax(e.vx + e.cf, vfs[1]), R(0));
        const R bm = fmin(fmin(e.vx - e.cf, vfs[0]), R(0));
        const R iden = frcp(bp - bm);
#pragma unroll
        for (int r = 0; r < 7; r++) cav[r] = (bp * F[0][r] - bm * F[1][r]) * iden + bp * bm * iden * (U[1][r] - U[0][r]);
    }
}

// Phase C.  Correction of a face from the limiter values of its two zones
// (gL of the left zone, gR of the right one): gamma_k, beta_k and
// sum_k beta_k R_k, assembled in (rho, v, B_t, P) and mapped to conserved
// variables once (7 frame rows).  The modified flux is
// cav - (dx / (2 dt)) c (face_combine).
// glim(k, gL, gR) yields the two limiter values of wave k.
template <typename R, typename GLim>
__device__ __forceinline__ void face_correction(GLim glim, const FaceEig<R>& e, const R alpha[7], const R nu[7],
                                                const Coef<R>& cf, R c[7]) {
#pragma clang fp contract(on)
    R bet[7];
#pragma unroll
    for (int k = 0; k < 7; k++) {
        R gL, gR;
        glim(k, gL, gR);
        R gk = (fabs(alpha[k]) > alpha_min(alpha[k])) ? gdiv(gR - gL, alpha[k]) : R(0);
        bet[k] = qvisc(nu[k] + gk, cf.eps[k], cf.q4e[k]) * alpha[k] - (gL + gR);
    }
    R bfp = bet[6] + bet[0], bfm = bet[6] - bet[0];
    R bsp = bet[4] + bet[2], bsm = bet[4] - bet[2];
    R bap = bet[5] + bet[1], bam = bet[5] - bet[1];
    R wrho = e.rho * (e.alf * bfp + e.als * bsp) + bet[3];
    R wvx = e.alf * e.cf * bfm + e.als * e.cs * bsm;
    R wvpar = e.s * (-e.als * e.cs * bfm + e.alf * e.cf * bsm);
    R wvy = wvpar * e.by - bap * e.bz;
    R wvz = wvpar * e.bz + bap * e.by;
    R wbpar = e.sq * e.a * (e.als * bfp - e.alf * bsp);
    R wb1 = wbpar * e.by + e.s * e.sq * bam * e.bz;
    R wb2 = wbpar * e.bz - e.s * e.sq * bam * e.by;
    R wp = e.rho * e.a2 * (e.alf * bfp + e.als * bsp);
    R v2 = e.vx * e.vx + e.vy * e.vy + e.vz * e.vz;
    c[0] = wrho;
    c[1] = e.vx * wrho + e.rho * wvx;
    c[2] = e.vy * wrho + e.rho * wvy;
    c[3] = e.vz * wrho + e.rho * wvz;
    c[4] = (R(0.5) * v2 + cf.gm2 * e.X * cf.igm1) * wrho + e.rho * (e.vx * wvx + e.vy * wvy + e.vz * wvz) +
           e.b1 * wb1 + e.b2 * wb2 + wp * cf.igm1;
    c[5] = wb1;
    c[6] = wb2;
}

template <typename R>
__device__ __forceinline__ void face_combine(const R cav[7], const R c[7], R il, R out[7]) {
#pragma clang fp contract(on)
#pragma unroll
    for (int r = 0; r < 7; r++) out[r] = cav[r] - il * c[r];
}

// the 7 frame rows of a face flux to the lab rows of direction D
template <typename R, int D>
__device__ __forceinline__ void store_flux(const R out[7], __amdgpu_buffer_rsrc_t rs, unsigned xo, unsigned fo,
                                           unsigned VB) {
    constexpr int A1 = (D + 1) % 3, A2 = (D + 2) % 3;
    // frame -> lab rows: m_par -> m_D, m_t1 -> m_A1, m_t2 -> m_A2
    bstore(out[0], rs, xo, fo);
    bstore(out[1], rs, xo, fo + (1 + D) * VB);
    bstore(out[2], rs, xo, fo + (1 + A1) * VB);
    bstore(out[3], rs, xo, fo + (1 + A2) * VB);
    bstore(out[4], rs, xo, fo + 4 * VB);
    bstore(out[5], rs, xo, fo + 5 * VB);
    bstore(out[6], rs, xo, fo + 6 * VB);
}

template <typename R, int D, int STAGE, bool MM, bool PROT>
__global__ void __launch_bounds__(1024) sweep_kernel(R* __restrict__ pool, const PatchDev* __restrict__ patches,
                                                     const WorkItem* __restrict__ work, DevParams prm, Coef<R> cf,
                                                     int cur, const StepConst* __restrict__ sc, int P, int W, int zlo,
                                                     unsigned long long* __restrict__ nprot) {
    extern __shared__ unsigned char smem_raw[];
    const int nthr = P * W;
    Rec8<R>* shp = reinterpret_cast<Rec8<R>*>(smem_raw);  // zone primitives
    Rec8<R>* shg = shp + nthr;                             // face g-tilde

    constexpr int FA = (D == 0) ? 1 : 0;                 // fast transverse axis
    constexpr int SA = (D == 0) ? 2 : (D == 1 ? 2 : 1);  // slow transverse axis
    constexpr unsigned ES = sizeof(R);

    const WorkItem wi = work[blockIdx.x];
    if (wi.patch < 0) return;  // padding item (whole block, before any barrier)
    const PatchDev Pt = patches[wi.patch];
    if (!Pt.active) return;  // frozen patch (whole block, before any barrier)
    // block (P, W) along x for D = x, (W, P) otherwise: consecutive lanes are
    // consecutive x either way
    const int s = (D == 0) ? (int)threadIdx.x : (int)threadIdx.y;
    const int w = (D == 0) ? (int)threadIdx.y : (int)threadIdx.x;
    const int tid = (D == 0) ? s + P * w : w + W * s;
    const int sstep = (D == 0) ? 1 : W;  // LDS distance between neighbours along the pencil
    const int pen = wi.a + w;            // pencil number in the item's rectangle
    const bool live = pen <= wi.c;
    // the item's rectangle of pencils in the transverse plane: tf pencils
    // along the fast axis from flo, rows along the slow axis from slo
    const int flo = (wi.b & 1023) - 512, slo = ((wi.b >> 10) & 1023) - 512, tf = wi.b >> 20;
    const int g = prm.ghost;
    // pen = slow * tf + fast; (pen + 1/2)/tf is at least 1/(2 tf) from an
    // integer, far above the error of the single-precision reciprocal
    const int slow = (int)(((float)pen + 0.5f) * __builtin_amdgcn_rcpf((float)tf));
    int zc[3];
    zc[D] = zlo + s;
    zc[FA] = flo + (pen - slow * tf);
    zc[SA] = slo + slow;
    const unsigned V = (unsigned)Pt.vol;
    const unsigned st[3] = {1u, (unsigned)Pt.N[0], (unsigned)(Pt.N[0] * Pt.N[1])};
    const unsigned x = live ? (unsigned)(zc[0] + g) + st[1] * (unsigned)(zc[1] + g) + st[2] * (unsigned)(zc[2] + g) : 0u;
    const unsigned xo = x * ES;  // zone byte offset (VGPR)
    const unsigned VB = V * ES;  // field byte stride (SGPR)
    const R lam = sc_lam(*sc, D, R(0));
    const __amdgpu_buffer_rsrc_t rs = patch_rsrc(pool + Pt.base, (unsigned)F_STATE * VB);     // state
    const __amdgpu_buffer_rsrc_t rw = patch_rsrc(pool + Pt.sbase, (unsigned)F_SCRATCH * VB);  // step intermediates
    const unsigned qs = (unsigned)(cur ? F_ST1 : F_ST0) * VB;  // state copy
    const R z0 = R(0);

    // ---------------- phase A: zone primitives ----------------
    if (live) {
        if (STAGE == 1 && D == 0) {
            // Step 2: reference EMF E^r = -v x B from q^n on [-3, n+2]^3
            if (zc[0] >= -3 && zc[0] <= Pt.n[0] + 2) {
                R u[8];
#pragma unroll
                for (int c = 0; c < 8; c++) u[c] = bload(z0, rs, xo, qs + c * VB);
                R ir = frcp(u[0]);
                R vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
                bstore(vz * u[5] - vy * u[6], rw, xo, (unsigned)F_ER * VB);
                bstore(vx * u[6] - vz * u[4], rw, xo, (unsigned)(F_ER + 1) * VB);
                bstore(vy * u[4] - vx * u[5], rw, xo, (unsigned)(F_ER + 2) * VB);
            }
        }
        shp[tid] = zone_phase<R, D, STAGE>(rs, rw, xo, st, qs, VB, cf, prm, *sc);
    }
    __syncthreads();

    // ---------------- phase B: face s between zones s-1 and s ----------------
    FaceEig<R> e;
    R alpha[7], nu[7];
    R bf = R(0);
    bool prot = false;
    const bool face = live && s >= 1;
    if (face) {
        bf = (STAGE == 1) ? bload(z0, rs, xo, qs + (8 + D) * VB) : bload(z0, rw, xo, (unsigned)(F_BH + D) * VB);
        Rec8<R> gr;
        face_phase<R, PROT>(shp[tid - sstep], shp[tid], bf, lam, cf, e, alpha, nu, gr, prot);
        shg[tid] = gr;
    }
    __syncthreads();

    // ---------------- phase C: modified flux at faces 2 .. P-2 ----------------
    if (face && s >= 2 && s <= P - 2) {
        R cav[7], out[7];
        if (PROT && prot) {
            face_central<R, PROT>(shp[tid - sstep], shp[tid], bf, e, prot, cf, out);
            atomicAdd(nprot, 1ULL);
        } else {
            const Rec8<R> Gm = shg[tid - sstep], G0 = shg[tid], Gp = shg[tid + sstep];
            R c[7];
            auto glim = [&](int k, R& gL, R& gR) {
                gL = sweby<MM>(G0.v[k], Gm.v[k], cf.beta_l);  // zone s-1: faces s-1 (left), s (right)
                gR = sweby<MM>(Gp.v[k], G0.v[k], cf.beta_l);  // zone s: faces s, s+1
            };
            face_correction<R>(glim, e, alpha, nu, cf, c);
            face_central<R, PROT>(shp[tid - sstep], shp[tid], bf, e, prot, cf, cav);
            face_combine(cav, c, sc_il(*sc, D, R(0)), out);
        }
        store_flux<R, D>(out, rw, xo, (unsigned)((STAGE == 1 ? F_FL1 : F_FL2) + 7 * D) * VB, VB);
    }
}

// ---------------------------------------------------------------------------
// Marching form of the y and z sweeps.  One thread owns one whole pencil
// along D and walks it zone by zone; the lanes of a wave hold consecutive
// pencils of the item's rectangle, numbered x fastest, so every load and
// store of a wave covers consecutive x.  The face and limiter data a later
// face needs are carried in registers from one zone to the next: zone s
// gives face s (phase B), whose g-tilde completes the limiter value of zone
// s-1 and with it the modified flux of face s-1 (phase C).  No LDS, no
// barrier; the same arithmetic as the pencil kernel, face by face.
// ---------------------------------------------------------------------------

template <typename R>
struct MarchFace {
    Rec8<R> rec;      // zone s
    FaceEig<R> e;     // face s (between zones s-1 and s)
    R alpha[7], nu[7], cav[7];
    Rec8<R> gt;       // g-tilde of face s
    R gz[7];          // limiter value of zone s-1
    bool prot;
};

template <typename R, int D, int STAGE, bool MM, bool PROT, bool PF2>
__global__ void __launch_bounds__(256) march_kernel(R* __restrict__ pool, const PatchDev* __restrict__ patches,
                                                    const WorkItem* __restrict__ work, DevParams prm, Coef<R> cf,
                                                    int cur, const StepConst* __restrict__ sc, int P, int zlo,
                                                    unsigned long long* __restrict__ nprot) {
    static_assert(D == 1 || D == 2, "the marching form serves the y and z sweeps");
    constexpr int SA = (D == 1) ? 2 : 1;  // slow transverse axis (x is the fast one)
    constexpr unsigned ES = sizeof(R);
    const WorkItem wi = work[blockIdx.x];
    if (wi.patch < 0) return;  // padding item
    const PatchDev Pt = patches[wi.patch];
    if (!Pt.active) return;  // frozen patch
    const int pen = wi.a + (int)threadIdx.x;
    if (pen > wi.c) return;  // past the item's last pencil (no barrier follows)
    const int flo = (wi.b & 1023) - 512, slo = ((wi.b >> 10) & 1023) - 512, tf = wi.b >> 20;
    const int g = prm.ghost;
    const int slow = (int)(((float)pen + 0.5f) * __builtin_amdgcn_rcpf((float)tf));
    int zc[3];
    zc[D] = zlo;
    zc[0] = flo + (pen - slow * tf);
    zc[SA] = slo + slow;
    const unsigned st[3] = {1u, (unsigned)Pt.N[0], (unsigned)(Pt.N[0] * Pt.N[1])};
    unsigned xo = ((unsigned)(zc[0] + g) + st[1] * (unsigned)(zc[1] + g) + st[2] * (unsigned)(zc[2] + g)) * ES;
    const unsigned sD = st[D] * ES;
    const unsigned VB = (unsigned)Pt.vol * ES;
    const StepConst scv = *sc;
    const R lam = sc_lam(scv, D, R(0)), il = sc_il(scv, D, R(0));
    const __amdgpu_buffer_rsrc_t rs = patch_rsrc(pool + Pt.base, (unsigned)F_STATE * VB);     // state
    const __amdgpu_buffer_rsrc_t rw = patch_rsrc(pool + Pt.sbase, (unsigned)F_SCRATCH * VB);  // step intermediates
    const __amdgpu_buffer_rsrc_t rb = (STAGE == 1) ? rs : rw;  // the face field B_D: b^n or b^{n+1/2}
    const unsigned qs = (unsigned)(cur ? F_ST1 : F_ST0) * VB;
    const unsigned bfo = (STAGE == 1) ? qs + (8 + D) * VB : (unsigned)(F_BH + D) * VB;
    const unsigned fo = (unsigned)((STAGE == 1 ? F_FL1 : F_FL2) + 7 * D) * VB;
    const R z0 = R(0);

    // Zone s's loads and face field requested one iteration ahead, so that
    // their latency overlaps the previous face's arithmetic: always in FP32
    // Step 1 (9 loads a zone) and in the FP32 corrector from stored records
    // (STAGE 3, 8 loads); in the FP32 corrector from q^n and the Step-1
    // fluxes (43 loads a zone) as the variant PF2, which takes 2 waves a
    // SIMD instead of 4; never in FP64, whose marching kernels already use
    // 256 VGPRs.
    constexpr bool PF = sizeof(R) == 4 && (STAGE != 2 || PF2);
    MarchFace<R> pv;  // zone s-1 and face s-1
    pv.rec = zone_phase<R, D, STAGE>(rs, rw, xo, st, qs, VB, cf, prm, scv);
    ZoneRaw<R, STAGE> nx;
    R bfn = R(0);
    if constexpr (PF) {
        zone_fetch<R, D, STAGE>(rs, rw, xo + sD, st, qs, VB, nx);
        bfn = bload(z0, rb, xo + sD, bfo);
    }
    for (int s = 1; s < P; s++) {
        xo += sD;
        MarchFace<R> cu;
        R bf;
        if constexpr (PF) {
            cu.rec = zone_record<R, D, STAGE>(nx, cf, prm, scv);
            bf = bfn;
            if (s + 1 < P) {
                zone_fetch<R, D, STAGE>(rs, rw, xo + sD, st, qs, VB, nx);
                bfn = bload(z0, rb, xo + sD, bfo);
            }
        } else {
            cu.rec = zone_phase<R, D, STAGE>(rs, rw, xo, st, qs, VB, cf, prm, scv);
            bf = bload(z0, rb, xo, bfo);
        }
        face_phase<R, PROT>(pv.rec, cu.rec, bf, lam, cf, cu.e, cu.alpha, cu.nu, cu.gt, cu.prot);
        if (s >= 2 && s <= P - 2) face_central<R, PROT>(pv.rec, cu.rec, bf, cu.e, cu.prot, cf, cu.cav);
        if (s >= 2) {
#pragma unroll
            for (int k = 0; k < 7; k++) cu.gz[k] = sweby<MM>(cu.gt.v[k], pv.gt.v[k], cf.beta_l);  // zone s-1
        }
        if (s >= 3) {
            // face s-1 (2 <= s-1 <= P-2): limiter values of zones s-2 and s-1
            R out[7];
            if (PROT && pv.prot) {
#pragma unroll
                for (int r = 0; r < 7; r++) out[r] = pv.cav[r];
                atomicAdd(nprot, 1ULL);
            } else {
                R c[7];
                auto glim = [&](int k, R& gL, R& gR) {
                    gL = pv.gz[k];
                    gR = cu.gz[k];
                };
                face_correction<R>(glim, pv.e, pv.alpha, pv.nu, cf, c);
                face_combine(pv.cav, c, il, out);
            }
            store_flux<R, D>(out, rw, xo - sD, fo, VB);
        }
        pv = cu;
    }
}

// ---------------------------------------------------------------------------
// Fused corrector (Steps 5-7 along x and y in one launch, and the z
// predictor records).  A block covers one z-plane k of a patch and a band of
// rows along y; every thread owns one zone (x fastest, so loads cover
// consecutive x), loads the zone's data once (q^n, b^n at the zone's lower
// and upper faces, the three Step-1 flux arrays at the zone and one zone up
// along their own axes) and builds from it the predictor states
// q^{n+1/2}_x, q^{n+1/2}_y and q^{n+1/2}_z (Step 5), which the separate
// sweeps each load and build on their own.  The x faces of the band's rows,
// then the y faces of the band, are formed as in the pencil kernel through
// the same LDS (zone records, then face g-tilde), with the same phase
// functions, so the fluxes are bitwise those of the separate sweeps.
//   block (P, RT): P = n_x + 6 zones [-3, n_x + 3) along x; RT rows along y,
//   the band's y-face rows [y0, y1) with two rows below and one above (the
//   limiter stencil); item a = k + XY_BIAS, b = (y0 + XY_BIAS) | (y1 +
//   XY_BIAS) << 16.
// x faces are formed on the band's rows within [-1, n_y], y faces on the
// band's rows at x in [-1, n_x]: the ranges of the separate sweeps.  The
// same loads also give the z predictor state of the band's rows at x in
// [-1, n_x]; its record (7 words) is stored in the zone's z corrector flux
// rows, where the z sweep then reads it (STAGE 3) instead of 43 loads of
// q^n and the Step-1 fluxes.  The z pencils need records on the planes
// [-3, n_z + 3): the items of the four planes beyond [-1, n_z] form only
// these records.
// ---------------------------------------------------------------------------

// rows of a transverse Step-1 flux in ZoneRaw's order (rows 0-4, then the
// row of B_D, then the other B row): for the first transverse axis A1 the
// B_D row is 6, for the second A2 it is 5
__device__ __forceinline__ constexpr int row_a1(int r) { return r < 5 ? r : (r == 5 ? 6 : 5); }
__device__ __forceinline__ constexpr int row_a2(int r) { return r < 5 ? r : (r == 5 ? 5 : 6); }

template <typename R, int D, bool MM, bool PROT>
__device__ __forceinline__ void xy_flux(const Rec8<R>* shp, const Rec8<R>* shg, int tid, int step, R bf,
                                        const FaceEig<R>& e, const R alpha[7], const R nu[7], bool prot,
                                        const Coef<R>& cf, R il, __amdgpu_buffer_rsrc_t rw, unsigned xo, unsigned VB,
                                        unsigned long long* nprot) {
    R out[7];
    if (PROT && prot) {
        face_central<R, PROT>(shp[tid - step], shp[tid], bf, e, prot, cf, out);
        atomicAdd(nprot, 1ULL);
    } else {
        const Rec8<R> Gm = shg[tid - step], G0 = shg[tid], Gp = shg[tid + step];
        R c[7], cav[7];
        auto glim = [&](int k, R& gL, R& gR) {
            gL = sweby<MM>(G0.v[k], Gm.v[k], cf.beta_l);
            gR = sweby<MM>(Gp.v[k], G0.v[k], cf.beta_l);
        };
        face_correction<R>(glim, e, alpha, nu, cf, c);
        face_central<R, PROT>(shp[tid - step], shp[tid], bf, e, prot, cf, cav);
        face_combine(cav, c, il, out);
    }
    store_flux<R, D>(out, rw, xo, (unsigned)(F_FL2 + 7 * D) * VB, VB);
}

// FP64 blocks stay within 512 threads (the LDS bound of the launch implies
// it), which leaves the FP64 kernel its 142 VGPRs without spilling.
template <typename R, bool MM, bool PROT>
__global__ void __launch_bounds__(sizeof(R) == 4 ? 1024 : 512)
    corr_xy_kernel(R* __restrict__ pool, const PatchDev* __restrict__ patches, const WorkItem* __restrict__ work,
                   DevParams prm, Coef<R> cf, int cur, const StepConst* __restrict__ sc,
                   unsigned long long* __restrict__ nprot) {
    extern __shared__ unsigned char smem_raw[];
    const int P = (int)blockDim.x, RT = (int)blockDim.y;
    Rec8<R>* shp = reinterpret_cast<Rec8<R>*>(smem_raw);  // zone records: x, then y
    Rec8<R>* shg = shp + P * RT;                          // face g-tilde: x, then y
    constexpr unsigned ES = sizeof(R);

    const WorkItem wi = work[blockIdx.x];
    if (wi.patch < 0) return;  // padding item (whole block, before any barrier)
    const PatchDev Pt = patches[wi.patch];
    if (!Pt.active) return;  // frozen patch (whole block, before any barrier)
    const int tx = (int)threadIdx.x, ty = (int)threadIdx.y, tid = tx + P * ty;
    const int k = wi.a - XY_BIAS;
    const int y0 = (wi.b & 0xffff) - XY_BIAS, y1 = (wi.b >> 16) - XY_BIAS;
    const int rows = y1 - y0 + 3;  // the band's rows, [y0 - 2, y1]
    const int x = tx - 3, y = y0 - 2 + ty;
    const bool live = ty < rows;
    const bool faces = k >= -1 && k <= Pt.n[2];  // planes of x and y faces (others: z records only)
    const bool own = live && y >= y0 && y < y1 && y <= Pt.n[1];     // the band's rows within [-1, n_y]
    const bool needX = faces && own;                                // x faces of this row
    const bool needY = faces && live && x >= -1 && x <= Pt.n[0];    // y faces of this column
    const bool needZ = own && x >= -1 && x <= Pt.n[0];              // the z predictor record
    const int g = prm.ghost;
    const unsigned st[3] = {1u, (unsigned)Pt.N[0], (unsigned)(Pt.N[0] * Pt.N[1])};
    const unsigned xo = live ? ((unsigned)(x + g) + st[1] * (unsigned)(y + g) + st[2] * (unsigned)(k + g)) * ES : 0u;
    const unsigned VB = (unsigned)Pt.vol * ES;
    const StepConst scv = *sc;
    const __amdgpu_buffer_rsrc_t rs = patch_rsrc(pool + Pt.base, (unsigned)F_STATE * VB);     // state
    const __amdgpu_buffer_rsrc_t rw = patch_rsrc(pool + Pt.sbase, (unsigned)F_SCRATCH * VB);  // step intermediates
    const unsigned qs = (unsigned)(cur ? F_ST1 : F_ST0) * VB;
    const R z0 = R(0);

    // ---------------- phase A: one load of the zone, three predictor records ----------------
    Rec8<R> ry;
    if (live) {
        ZoneRaw<R, 2> zx, zy;
#pragma unroll
        for (int c = 0; c < 8; c++) zx.q[c] = zy.q[c] = bload(z0, rs, xo, qs + c * VB);
        const unsigned bs = qs + 8 * VB;
#pragma unroll
        for (int a = 0; a < 3; a++) {
            zx.b[a][0] = zy.b[a][0] = bload(z0, rs, xo, bs + a * VB);
            zx.b[a][1] = zy.b[a][1] = bload(z0, rs, xo, bs + a * VB + st[a] * ES);
        }
        R F[3][7][2];  // Step-1 fluxes along x, y, z at the zone and one zone up along their axis
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int r = 0; r < 7; r++) {
                const unsigned fo = (unsigned)(F_FL1 + 7 * a + r) * VB;
                F[a][r][0] = bload(z0, rw, xo, fo);
                F[a][r][1] = bload(z0, rw, xo, fo + st[a] * ES);
            }
        // x predictor: transverse axes y (A1) and z (A2); y predictor: z (A1) and x (A2)
#pragma unroll
        for (int r = 0; r < 7; r++)
#pragma unroll
            for (int s = 0; s < 2; s++) {
                zx.fa[r][s] = F[1][row_a1(r)][s];
                zx.fb[r][s] = F[2][row_a2(r)][s];
                zy.fa[r][s] = F[2][row_a1(r)][s];
                zy.fb[r][s] = F[0][row_a2(r)][s];
            }
        if (needZ) {
            // z predictor: transverse axes x (A1) and y (A2); its record goes
            // to the z corrector flux rows, which the z sweep (STAGE 3) reads
            ZoneRaw<R, 2> zz;
#pragma unroll
            for (int c = 0; c < 8; c++) zz.q[c] = zx.q[c];
#pragma unroll
            for (int a = 0; a < 3; a++) zz.b[a][0] = zx.b[a][0], zz.b[a][1] = zx.b[a][1];
#pragma unroll
            for (int r = 0; r < 7; r++)
#pragma unroll
                for (int s2 = 0; s2 < 2; s2++) {
                    zz.fa[r][s2] = F[0][row_a1(r)][s2];
                    zz.fb[r][s2] = F[1][row_a2(r)][s2];
                }
            const Rec8<R> rz = zone_record<R, 2, 2>(zz, cf, prm, scv);
#pragma unroll
            for (int r = 0; r < 7; r++) bstore(rz.v[r], rw, xo, (unsigned)(F_FL2 + 14 + r) * VB);
        }
        // the z record first (stored at once), so that its temporaries are
        // dead before the x and y records are formed
        __builtin_amdgcn_sched_barrier(0);
        if (needX) shp[tid] = zone_record<R, 0, 2>(zx, cf, prm, scv);
        if (needY) ry = zone_record<R, 1, 2>(zy, cf, prm, scv);
    }
    if (!faces) return;  // a z-record plane: no barrier follows for the whole block
    __syncthreads();

    // ---------------- x faces: tx - 3 between zones tx - 4 and tx - 3 ----------------
    {
        FaceEig<R> e;
        R alpha[7], nu[7];
        R bf = R(0);
        bool prot = false;
        const bool face = needX && tx >= 1;
        if (face) {
            bf = bload(z0, rw, xo, (unsigned)F_BH * VB);
            Rec8<R> gr;
            face_phase<R, PROT>(shp[tid - 1], shp[tid], bf, sc_lam(scv, 0, R(0)), cf, e, alpha, nu, gr, prot);
            shg[tid] = gr;
        }
        __syncthreads();
        if (face && tx >= 2 && tx <= P - 2)
            xy_flux<R, 0, MM, PROT>(shp, shg, tid, 1, bf, e, alpha, nu, prot, cf, sc_il(scv, 0, R(0)), rw, xo, VB,
                                    nprot);
    }
    __syncthreads();  // the x records and g-tilde are read
    if (needY) shp[tid] = ry;
    __syncthreads();

    // ---------------- y faces: y between rows ty - 1 and ty ----------------
    {
        FaceEig<R> e;
        R alpha[7], nu[7];
        R bf = R(0);
        bool prot = false;
        const bool face = needY && ty >= 1;
        if (face) {
            bf = bload(z0, rw, xo, (unsigned)(F_BH + 1) * VB);
            Rec8<R> gr;
            face_phase<R, PROT>(shp[tid - P], shp[tid], bf, sc_lam(scv, 1, R(0)), cf, e, alpha, nu, gr, prot);
            shg[tid] = gr;
        }
        __syncthreads();
        if (face && ty >= 2 && ty <= rows - 2)
            xy_flux<R, 1, MM, PROT>(shp, shg, tid, P, bf, e, alpha, nu, prot, cf, sc_il(scv, 1, R(0)), rw, xo, VB,
                                    nprot);
    }
}

// ---------------------------------------------------------------------------
// FP64 diagnostics with compensated sums.  Every running sum is an unevaluated
// pair hi + lo: a value is added with the error-free TwoSum, and two pairs
// are merged by adding their high parts error-free and their low parts
// plainly, then renormalising.  The result is accurate to about one rounding
// of the exact sum, whatever the order, and the order itself is fixed (the
// reduction trees below do not depend on timing), so results are bitwise
// reproducible.
//   diag_kernel        one block per work item (a run of interior zones of one
//                      patch): per thread TwoSum accumulation, then a fixed
//                      butterfly across the wave and a fixed merge of the waves;
//                      writes one record of DIAG_REC doubles per item
//   diag_final_kernel  one wave: merges the records in item order into the
//                      totals, B_rms, the max of |div b| and the counters
// ---------------------------------------------------------------------------

constexpr int DIAG_NSUM = 9;   // q (8) times the zone volume, |B|^2
constexpr int DIAG_THREADS = 256;

struct DSum {
    double hi, lo;
};

__device__ __forceinline__ void two_sum_add(DSum& a, double x) {
#pragma clang fp contract(off)
    const double s = a.hi + x;
    const double bb = s - a.hi;
    const double err = (a.hi - (s - bb)) + (x - bb);
    a.hi = s;
    a.lo += err;
}

__device__ __forceinline__ DSum merge(DSum a, DSum b) {
#pragma clang fp contract(off)
    DSum r{a.hi, a.lo + b.lo};
    two_sum_add(r, b.hi);
    const double h = r.hi + r.lo;  // renormalise (|lo| is far below |hi|)
    r.lo = r.lo - (h - r.hi);
    r.hi = h;
    return r;
}

__device__ __forceinline__ DSum shfl_xor_dsum(DSum a, int off) {
    return DSum{__shfl_xor(a.hi, off, 64), __shfl_xor(a.lo, off, 64)};
}

template <typename R>
__global__ void __launch_bounds__(DIAG_THREADS) diag_kernel(const R* __restrict__ pool, const PatchDev* __restrict__ patches,
                                                            const WorkItem* __restrict__ work, DevParams prm, int cur,
                                                            double* __restrict__ rec) {
#pragma clang fp contract(off)
    __shared__ double red[DIAG_THREADS / 64][2 * DIAG_NSUM + 1];
    const WorkItem w = work[blockIdx.x];  // a = first interior zone (linear, x fastest), b = zone count
    const PatchDev P = patches[w.patch];
    const int g = prm.ghost;
    const long long V = P.vol;
    const R* q = pool + P.base + (long long)(cur ? F_ST1 : F_ST0) * V;
    const R* b = q + 8 * V;
    const double dV = prm.dx[0] * prm.dx[1] * prm.dx[2];
    DSum acc[DIAG_NSUM];
#pragma unroll
    for (int c = 0; c < DIAG_NSUM; c++) acc[c] = DSum{0.0, 0.0};
    double mx = 0.0;
    const int zend = P.present ? w.a + w.b : w.a;  // an absent slot adds nothing
    for (int z = w.a + (int)threadIdx.x; z < zend; z += DIAG_THREADS) {
        const int i = z % P.n[0], t = z / P.n[0];
        const int j = t % P.n[1], k = t / P.n[1];
        const long long x = sidx(P, i + g, j + g, k + g);
#pragma unroll
        for (int c = 0; c < 8; c++) two_sum_add(acc[c], (double)q[(long long)c * V + x] * dV);
        const double b0 = q[4 * V + x], b1 = q[5 * V + x], b2 = q[6 * V + x];
        two_sum_add(acc[8], b0 * b0 + b1 * b1 + b2 * b2);
        double div = 0.0;
#pragma unroll
        for (int d = 0; d < 3; d++)
            div += ((double)b[(long long)d * V + x + stride_of(P, d)] - (double)b[(long long)d * V + x]) / prm.dx[d];
        mx = fmax(mx, fabs(div));
    }
    // butterfly across the wave (every lane ends with the same merged value)
    for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
        for (int c = 0; c < DIAG_NSUM; c++) acc[c] = merge(acc[c], shfl_xor_dsum(acc[c], off));
        mx = fmax(mx, __shfl_xor(mx, off, 64));
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < DIAG_NSUM; c++) {
            red[wid][2 * c] = acc[c].hi;
            red[wid][2 * c + 1] = acc[c].lo;
        }
        red[wid][2 * DIAG_NSUM] = mx;
    }
    __syncthreads();
    if (threadIdx.x < DIAG_NSUM) {
        const int c = threadIdx.x;
        DSum s{red[0][2 * c], red[0][2 * c + 1]};
        for (int v = 1; v < DIAG_THREADS / 64; v++) s = merge(s, DSum{red[v][2 * c], red[v][2 * c + 1]});
        rec[(long long)blockIdx.x * DIAG_REC + 2 * c] = s.hi;
        rec[(long long)blockIdx.x * DIAG_REC + 2 * c + 1] = s.lo;
    } else if (threadIdx.x == DIAG_NSUM) {
        double m = red[0][2 * DIAG_NSUM];
        for (int v = 1; v < DIAG_THREADS / 64; v++) m = fmax(m, red[v][2 * DIAG_NSUM]);
        rec[(long long)blockIdx.x * DIAG_REC + 2 * DIAG_NSUM] = m;
        rec[(long long)blockIdx.x * DIAG_REC + 2 * DIAG_NSUM + 1] = 0.0;
    }
}

// out[0..7] totals, [8] max normalised div b, [9] max |div b|, [10] floor
// activations, [11] protected faces (counts as exact doubles)
__global__ void __launch_bounds__(64) diag_final_kernel(const double* __restrict__ rec, int nrec,
                                                         const unsigned long long* __restrict__ counters, double nzones,
                                                         double dmin, double* __restrict__ out) {
    const int lane = threadIdx.x;
    DSum acc[DIAG_NSUM];
#pragma unroll
    for (int c = 0; c < DIAG_NSUM; c++) acc[c] = DSum{0.0, 0.0};
    double mx = 0.0;
    for (int r = lane; r < nrec; r += 64) {
        const double* p = rec + (long long)r * DIAG_REC;
#pragma unroll
        for (int c = 0; c < DIAG_NSUM; c++) acc[c] = merge(acc[c], DSum{p[2 * c], p[2 * c + 1]});
        mx = fmax(mx, p[2 * DIAG_NSUM]);
    }
    for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
        for (int c = 0; c < DIAG_NSUM; c++) acc[c] = merge(acc[c], shfl_xor_dsum(acc[c], off));
        mx = fmax(mx, __shfl_xor(mx, off, 64));
    }
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < 8; c++) out[c] = acc[c].hi + acc[c].lo;
        double brms = sqrt((acc[8].hi + acc[8].lo) / (nzones > 0.0 ? nzones : 1.0));
        if (brms < 1e-300) brms = 1e-300;
        out[8] = mx * dmin / brms;
        out[9] = mx;
        out[10] = (double)counters[0];
        out[11] = (double)counters[1];
    }
}

// ---------------------------------------------------------------------------
// host-side launch wrappers
// ---------------------------------------------------------------------------

// the passes in mask (1: x, 2: y, 4: z), in that order
template <typename R>
hipError_t launch_fill(void* pool, const PatchDev* pt, const WorkItem* const wl[3], const int nw[3], int g, int cur,
                       int mask, hipStream_t st) {
    if ((mask & 1) && nw[0] > 0)
        hipLaunchKernelGGL((fill_pass_kernel<R, 0>), dim3(nw[0]), dim3(256), 0, st, (R*)pool, pt, wl[0], g, cur);
    if ((mask & 2) && nw[1] > 0)
        hipLaunchKernelGGL((fill_pass_kernel<R, 1>), dim3(nw[1]), dim3(256), 0, st, (R*)pool, pt, wl[1], g, cur);
    if ((mask & 4) && nw[2] > 0)
        hipLaunchKernelGGL((fill_pass_kernel<R, 2>), dim3(nw[2]), dim3(256), 0, st, (R*)pool, pt, wl[2], g, cur);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_dt_reduce(void* pool, const PatchDev* pt, const WorkItem* wk, int nblk, const DevParams& prm, int cur,
                            unsigned long long* smax, hipStream_t st) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, st, smax);
    if (nblk > 0) hipLaunchKernelGGL(dt_reduce_kernel<R>, dim3(nblk), dim3(256), 0, st, (const R*)pool, pt, wk, prm, cur, smax);
    return hipGetLastError();
}

hipError_t launch_dt_finalize(unsigned long long* smax, StepConst* sc, const DevParams& prm, hipStream_t st) {
    hipLaunchKernelGGL(dt_finalize_kernel, dim3(1), dim3(1), 0, st, smax, sc, prm);
    return hipGetLastError();
}

// one entry of the device patch table, ordered on the stream (freeze, thaw,
// removal and addition of patches between steps)
__global__ void set_patch_kernel(PatchDev* __restrict__ table, int idx, PatchDev v) {
    if (threadIdx.x == 0) table[idx] = v;
}

hipError_t launch_set_patch(PatchDev* table, int idx, const PatchDev& v, hipStream_t st) {
    hipLaunchKernelGGL(set_patch_kernel, dim3(1), dim3(64), 0, st, table, idx, v);
    return hipGetLastError();
}

hipError_t launch_set_dt(StepConst* sc, double dt, const DevParams& prm, hipStream_t st) {
    hipLaunchKernelGGL(set_dt_kernel, dim3(1), dim3(1), 0, st, sc, dt, prm);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_ct_half(void* pool, const PatchDev* pt, const WorkItem* wk, int nblk, const Coef<R>& cf, int g, int cur,
                          const StepConst* sc, hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(ct_half_kernel<R>, dim3(nblk), dim3(TILE_THREADS), 0, st, (R*)pool, pt, wk, cf, g, cur, sc);
    return hipGetLastError();
}

// queue != nullptr: the persistent form, with as many blocks as are
// resident at once (a multiple of 8), over a list of nblk items (a multiple
// of 8, as xcd_order pads it); queue holds 9 counters, zero between launches
template <typename R>
hipError_t launch_update(void* pool, const PatchDev* pt, const WorkItem* wk, int nblk, const DevParams& prm,
                         const Coef<R>& cf, int cur, const StepConst* sc, unsigned long long* nfl, unsigned long long* smax,
                         int keep_edges, int threads, unsigned int* queue, hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    if (threads < 64 || threads > UpdTile<R>::threads || threads % 64) return hipErrorInvalidValue;
    if (!queue) {
        hipLaunchKernelGGL((update_kernel<R, false>), dim3(nblk), dim3(threads), 0, st, (R*)pool, pt, wk, nblk, queue,
                           prm, cf, cur, sc, nfl, smax, keep_edges);
        return hipGetLastError();
    }
    if (nblk % 8) return hipErrorInvalidValue;
    int dev = 0, per_cu = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)update_kernel<R, true>, threads, 0);
    if (e != hipSuccess) return e;
    int grid = per_cu * cus;
    grid -= grid % 8;
    if (grid < 8) grid = 8;
    if (grid > nblk) grid = nblk;
    hipLaunchKernelGGL((update_kernel<R, true>), dim3(grid), dim3(threads), 0, st, (R*)pool, pt, wk, nblk, queue, prm,
                       cf, cur, sc, nfl, smax, keep_edges);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_sweep(int d, int stage, void* pool, const PatchDev* pt, const WorkItem* wk, int nblk, const DevParams& prm,
                        const Coef<R>& cf, int cur, const StepConst* sc, int P, int W, int zlo,
                        unsigned long long* nprot, hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    size_t shmem = sizeof(R) * 16 * (size_t)P * W;
    dim3 blk = (d == 0) ? dim3(P, W) : dim3(W, P);
    const bool mm = cf.beta_l == R(1);
    const bool pr = cf.rho_prot > R(0) || cf.p_prot > R(0);
#define WMB_SW1(DD, SS, MM, PR)                                                                                       \
    hipLaunchKernelGGL((sweep_kernel<R, DD, SS, MM, PR>), dim3(nblk), blk, shmem, st, (R*)pool, pt, wk, prm, cf, cur, sc, \
                       P, W, zlo, nprot)
#define WMB_SW(DD, SS)                                                                                                \
    do {                                                                                                              \
        if (mm && !pr) WMB_SW1(DD, SS, true, false);                                                                  \
        else if (mm) WMB_SW1(DD, SS, true, true);                                                                     \
        else if (!pr) WMB_SW1(DD, SS, false, false);                                                                  \
        else WMB_SW1(DD, SS, false, true);                                                                            \
    } while (0)
    if (stage == 3) {
        if (d != 2) return hipErrorInvalidValue;  // the z corrector from stored records
        WMB_SW(2, 3);
    } else if (stage == 1) {
        if (d == 0) WMB_SW(0, 1);
        else if (d == 1) WMB_SW(1, 1);
        else WMB_SW(2, 1);
    } else {
        if (d == 0) WMB_SW(0, 2);
        else if (d == 1) WMB_SW(1, 2);
        else WMB_SW(2, 2);
    }
#undef WMB_SW1
#undef WMB_SW
    return hipGetLastError();
}

// diagnostics into out[12] (device memory); rec holds nblk records of DIAG_REC doubles
// the marching y/z sweeps: W threads (pencils) a block
template <typename R>
hipError_t launch_march(int d, int stage, void* pool, const PatchDev* pt, const WorkItem* wk, int nblk, const DevParams& prm,
                        const Coef<R>& cf, int cur, const StepConst* sc, int P, int W, int zlo,
                        unsigned long long* nprot, hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    // W > 512: the corrector with the one-zone-ahead loads (FP32), W - 512 pencils a block
    // (stage 3, the corrector from stored records, issues them ahead always in FP32)
    const bool pf = W > 512 && sizeof(R) == 4 && stage == 2;
    if (W > 512) W -= 512;
    if (d < 1 || d > 2 || W < 1 || W > 256) return hipErrorInvalidValue;
    const bool mm = cf.beta_l == R(1);
    const bool pr = cf.rho_prot > R(0) || cf.p_prot > R(0);
#define WMB_MA1(DD, SS, MM, PR)                                                                                     \
    do {                                                                                                            \
        if (pf)                                                                                                     \
            hipLaunchKernelGGL((march_kernel<R, DD, SS, MM, PR, true>), dim3(nblk), dim3(W), 0, st, (R*)pool, pt, wk, \
                               prm, cf, cur, sc, P, zlo, nprot);                                                    \
        else                                                                                                        \
            hipLaunchKernelGGL((march_kernel<R, DD, SS, MM, PR, false>), dim3(nblk), dim3(W), 0, st, (R*)pool, pt,    \
                               wk, prm, cf, cur, sc, P, zlo, nprot);                                                \
    } while (0)
#define WMB_MA3(MM, PR)                                                                                             \
    hipLaunchKernelGGL((march_kernel<R, 2, 3, MM, PR, false>), dim3(nblk), dim3(W), 0, st, (R*)pool, pt, wk, prm,   \
                       cf, cur, sc, P, zlo, nprot)
#define WMB_MA(DD, SS)                                                                                              \
    do {                                                                                                            \
        if (mm && !pr) WMB_MA1(DD, SS, true, false);                                                                \
        else if (mm) WMB_MA1(DD, SS, true, true);                                                                   \
        else if (!pr) WMB_MA1(DD, SS, false, false);                                                                \
        else WMB_MA1(DD, SS, false, true);                                                                          \
    } while (0)
    if (stage == 3) {
        // the z corrector from stored records (its loads always one zone ahead in FP32)
        if (d != 2) return hipErrorInvalidValue;
        if (mm && !pr) WMB_MA3(true, false);
        else if (mm) WMB_MA3(true, true);
        else if (!pr) WMB_MA3(false, false);
        else WMB_MA3(false, true);
    } else if (stage == 1) {
        if (d == 1) WMB_MA(1, 1);
        else WMB_MA(2, 1);
    } else {
        if (d == 1) WMB_MA(1, 2);
        else WMB_MA(2, 2);
    }
#undef WMB_MA1
#undef WMB_MA3
#undef WMB_MA
    return hipGetLastError();
}

// the fused x and y correctors: blocks of P = n_x + 6 by RT rows (one z-plane band each)
template <typename R>
hipError_t launch_corr_xy(void* pool, const PatchDev* pt, const WorkItem* wk, int nblk, const DevParams& prm,
                          const Coef<R>& cf, int cur, const StepConst* sc, int P, int RT, unsigned long long* nprot,
                          hipStream_t st) {
    if (nblk <= 0) return hipSuccess;
    // FP64 blocks stay within 512 threads (the kernel's launch bound), which the LDS bound implies
    if (P < 1 || RT < 4 || P * RT > 1024 || sizeof(R) * 16 * (size_t)P * RT > 64 * 1024) return hipErrorInvalidValue;
    const size_t shmem = sizeof(R) * 16 * (size_t)P * RT;
    const bool mm = cf.beta_l == R(1);
    const bool pr = cf.rho_prot > R(0) || cf.p_prot > R(0);
#define WMB_XY(MM, PR)                                                                                              \
    hipLaunchKernelGGL((corr_xy_kernel<R, MM, PR>), dim3(nblk), dim3(P, RT), shmem, st, (R*)pool, pt, wk, prm, cf, \
                       cur, sc, nprot)
    if (mm && !pr) WMB_XY(true, false);
    else if (mm) WMB_XY(true, true);
    else if (!pr) WMB_XY(false, false);
    else WMB_XY(false, true);
#undef WMB_XY
    return hipGetLastError();
}

template <typename R>
hipError_t launch_diag(const void* pool, const PatchDev* pt, const WorkItem* wk, int nblk, const DevParams& prm, int cur,
                       double* rec, const unsigned long long* counters, double nzones, double dmin, double* out,
                       hipStream_t st) {
    if (nblk > 0)
        hipLaunchKernelGGL(diag_kernel<R>, dim3(nblk), dim3(DIAG_THREADS), 0, st, (const R*)pool, pt, wk, prm, cur, rec);
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(64), 0, st, rec, nblk, counters, nzones, dmin, out);
    return hipGetLastError();
}

// explicit instantiations
#define WMB_INST(R)                                                                                                      \
    template hipError_t launch_fill<R>(void*, const PatchDev*, const WorkItem* const[3], const int[3], int, int, int,  \
                                       hipStream_t);                                                                     \
    template hipError_t launch_dt_reduce<R>(void*, const PatchDev*, const WorkItem*, int, const DevParams&, int,         \
                                            unsigned long long*, hipStream_t);                                           \
    template hipError_t launch_ct_half<R>(void*, const PatchDev*, const WorkItem*, int, const Coef<R>&, int, int,        \
                                          const StepConst*, hipStream_t);                                                \
    template hipError_t launch_update<R>(void*, const PatchDev*, const WorkItem*, int, const DevParams&, const Coef<R>&, \
                                         int, const StepConst*, unsigned long long*, unsigned long long*, int, int,     \
                                         unsigned int*, hipStream_t);                                                    \
    template hipError_t launch_sweep<R>(int, int, void*, const PatchDev*, const WorkItem*, int, const DevParams&,        \
                                        const Coef<R>&, int, const StepConst*, int, int, int, unsigned long long*,       \
                                        hipStream_t);                                                                    \
    template hipError_t launch_march<R>(int, int, void*, const PatchDev*, const WorkItem*, int, const DevParams&,        \
                                        const Coef<R>&, int, const StepConst*, int, int, int, unsigned long long*,       \
                                        hipStream_t);                                                                    \
    template hipError_t launch_corr_xy<R>(void*, const PatchDev*, const WorkItem*, int, const DevParams&,           \
                                          const Coef<R>&, int, const StepConst*, int, int, unsigned long long*,         \
                                          hipStream_t);                                                                  \
    template hipError_t launch_diag<R>(const void*, const PatchDev*, const WorkItem*, int, const DevParams&, int,        \
                                       double*, const unsigned long long*, double, double, double*, hipStream_t);
WMB_INST(float)
WMB_INST(double)
#undef WMB_INST

}  // namespace wmb
