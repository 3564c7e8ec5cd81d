// wmb_internal.h -- device-side layout shared by the runtime and the kernels
// of the patch MHD library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace wmb {

// Scheme parameters as the kernels see them.
struct DevParams {
    double gamma;
    double cfl;
    double eps[7];
    double limiter_beta;
    double rho_floor;
    double p_floor;
    double dx[3];
    double degen_tol;
    int ghost;
    int dt_lag;  // 1: dt of a step from the signal-speed maximum of the state one step earlier
};

// Per-step constants derived from dt, written on the device by the dt
// finalize kernel (or by the explicit-dt setter), read by every step kernel.
struct StepConst {
    double dt, hdt;
    double lam[3];  // dt / dx_d
    double il[3];   // dx_d / (2 dt)
    float fdt, fhdt;
    float flam[3];
    float fil[3];
};

// Scheme constants in the working precision, derived on the host once.
template <typename R>
struct Coef {
    R gam, gm1, gm2, ggm, igm1;  // gamma, gamma-1, gamma-2, gamma/(gamma-1), 1/(gamma-1)
    R beta_l, p_floor, rho_floor, tol, tol2;
    R idx[3];                    // 1 / dx_d
    R eps[7], q4e[7];            // epsilon_k and 1/(4 epsilon_k) (0 where epsilon_k = 0)
    R rho_prot, p_prot;          // protection floors (0: off)
};

// One patch inside the device pool: structure of arrays over the ghosted box
// N = n + 2g, x fastest.  Every field array holds `vol` elements starting at
// base + field * vol (elements of the working precision).
struct PatchDev {
    int n[3];
    int N[3];
    int nb[6];   // face neighbours: -x, +x, -y, +y, -z, +z (-1: domain boundary)
    int active;  // 0: frozen (no kernel updates it; its state is the same in both copies)
    int present; // 0: the slot is absent from the domain (removed: no neighbour links to it,
                 //    no kernel reads or writes it; also inactive)
    long long base;   // the patch's state region in the pool (words)
    long long sbase;  // its step intermediates (words; shared with the patches of
                      // other scratch groups, whose steps run at other times)
    long long vol;
};

// Field slots of a patch, in units of vol: the state region (kept between
// steps) ...
enum : int {
    F_ST0 = 0,   // state copy 0: q (8) then b (3)
    F_ST1 = 11,  // state copy 1
    F_STATE = 22
};
// ... and the step's intermediates (written and read within one step).
enum : int {
    F_FL1 = 0,   // Step-1 fluxes, 3 directions x 7 rows
    F_FL2 = 21,  // Step-6/7 fluxes, 3 directions x 7 rows
    F_ED = 42,   // edge EMFs (3), reused by Steps 3 and 9
    F_BH = 45,   // b^{n+1/2} (3)
    F_ER = 48,   // zone-centred reference EMF (3), reused by Steps 2 and 8
    F_SCRATCH = 51
};
// Row order of a flux array of direction d: rho, mx, my, mz, E, B_{d+1}, B_{d+2}
// (the B_d row of the 1D flux is identically zero and is not stored).

struct WorkItem {
    int patch;
    int a;  // box kernels: block index in the patch; sweeps: first pencil of the block
            // (numbered fast-transverse first within the item's rectangle);
            // tiles: i0 | j0 << 16 (biased)
    int b;  // sweeps: the pencil rectangle, (flo + 512) | (slo + 512) << 10 | fcnt << 20
            // (first fast and slow transverse coords, pencils along fast);
            // tiles: tx | ty << 16
    int c;  // sweeps: last pencil (inclusive); tiles: k0 | k1 << 16 (biased, k1 exclusive)
};

// Fused x/y corrector items (one z-plane band of a patch): a = k + XY_BIAS,
// b = (y0 + XY_BIAS) | (y1 + XY_BIAS) << 16 for the band's y-face rows
// [y0, y1) (plane k and rows may be -1).
constexpr int XY_BIAS = 16;

// Diagnostics record of one work item (doubles): 9 compensated sums as (hi, lo)
// pairs (q times the zone volume, |B|^2), the max |div b|, one pad word.
constexpr int DIAG_REC = 20;

// Column tiles of the Steps 8-11 kernel: the largest tile plane (one thread a
// zone, the block size).  FP32 may take 512 (fewer ring zones of E^r per tile
// zone at the same occupancy) where the patches' tiles fill such blocks; FP64
// (about 150 VGPRs) keeps 256, which lets three blocks share a CU where a
// 512-thread block would run alone.
constexpr int upd_tile_zones_max(int esize) { return esize == 4 ? 512 : 256; }

// The Steps 8-11 kernel's LDS planes, sized for its largest block: E^r over
// the tile and a one-zone ring, (tx + 2)(ty + 2) <= upd_er_plane, and the
// edges, (tx + 1)(ty + 1) <= upd_ed_plane.  The tile planner keeps every tile
// within both (and tx ty within the block).
constexpr int upd_er_plane(int esize) { return upd_tile_zones_max(esize) + 68 + upd_tile_zones_max(esize) / 16; }
constexpr int upd_ed_plane(int esize) { return upd_tile_zones_max(esize) + 33 + upd_tile_zones_max(esize) / 32; }

// Box kernels: interior-relative inclusive ranges [lo, n + hi] per axis.
struct Box {
    int lo, hi;
};

}  // namespace wmb
