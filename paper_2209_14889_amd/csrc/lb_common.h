// Shared host/device layout of liblb (MI355X, gfx950).  Plain structs of device pointers and
// coefficients; the host builds them once in lb_create and kernels read them from the arena.
#pragma once
#include <stdint.h>

namespace lbk {

constexpr int kMaxNodes = 1024;     // nodes per body
constexpr int kMaxBodies = 64;      // bodies per simulation
constexpr int kPatchTile = 16;      // immersed-boundary gather block: 16 x 16 patch sites
constexpr int kIbOneLaunchTiles = 512;   // up to this many patch tiles: body update in one launch
constexpr int kItemBodies = 8;      // bodies listed per fused work item (more: scan all of them)
constexpr int kBodyOut = 8;         // doubles per body written by the observable kernel
constexpr int kMaxCand = 512;       // nodes whose footprint can reach one gather block
constexpr int kStiffSeg = 64;       // stiffness-table segments over s = |P|^2 in [0, P_clamp^2]
constexpr int kHalo = 4;            // fused kernel: polarization halo depth (stress and h use 3)
constexpr int kDefaultShift = 10;   // FP16 storage: offsets scaled by 2^10

// status bits raised by kernels, read by the host at synchronising calls
constexpr int kStatusPatch = 1;     // a body outgrew its force/velocity patch
constexpr int kStatusUnstable = 2;  // watchdog: non-finite or drifting mass
constexpr int kStatusWall = 4;      // a node's kernel footprint reached a wall

struct SimDev {
    int nx, ny;
    int nb, b0;                     // bodies of this simulation: count, first index
    float omega, guo;               // 1/tau and 1 - 1/(2 tau)  (BGK, Guo forcing)
    float inv_eta, D;               // 1/eta_p, D_p
    float xi, alpha, beta, kappa, Gamma;
    float cA8, cA2, cB2;            // cA / 8, cA / 2, cB / 2 with cA = K1111-2K1122-4K1212+K2222,
                                    // cB = K1111-K2222 (the anisotropic parts of C~)
    float s1, s2, s3;               // isotropic parts: (3K1111+2K1122+4K1212+3K2222) / 8,
                                    // (K1111+6K1122-4K1212+K2222) / 8, (K1111-2K1122+4K1212+K2222) / 4
    float kap4;                     // kappa / 4 (the Ericksen gradient term from half-differences)
    float m4D, gk;                  // -4 D_p and Gamma kappa: the centre weight of the stress
                                    // Laplacian and the Laplacian weight of the P right-hand side
    float smax, inv_ds;             // table range P_clamp^2 and intervals per unit s
    float A2max, A4max;             // a2/s and a4/s^2 at smax
    float inv_scale, scale;         // FP16 storage scale 2^-S and 2^S (1 for FP32)
    int ericksen;
    int walls;                      // 1: bounce-back walls below row 0 and above row ny-1
    float gx, gy;                   // uniform body force
    const float *tab;               // per segment 8 floats: cubics in the local coordinate of A2 = a2/s, A4 = a4/s^2
    void *h[2];                     // post-collision population offsets, 9 planes (float or half)
    float *sig[2];                  // polymer stress planes sxx, syy, sxy
    void *P[2];                     // polarization planes, offsets Px - pref[0], Py - pref[1]: FP32
                                    // with FP16 populations, FP64 (pref = 0) with FP32 populations
    float pref[2];                  // reference polarization the offsets are taken from (FP32 form:
                                    // the mean of the initial field, rounded to FP32)
    double pref_d[2];               // the same in FP64, and alpha, beta in FP64 (the slope of the
    double alpha_d, beta_d;         // molecular field)
    float *sE;                      // scratch: Ericksen stress xx, xy, yx, yy
    float *v;                       // multi-pass scratch: velocity
    float *sps;                     // multi-pass scratch: predicted stress (3 planes)
    void *spp;                      // multi-pass scratch: predicted polarization offsets (2 planes)
};

struct BodyDev {
    int sim, n, ps, nside;          // owning sim, nodes, patch side, gather blocks per side
    double k, eps, leq, fx, fy, t_on, t_off, width;
    double trap_k, trap_x0, trap_y0, trap_dx, trap_dy, trap_t1, trap_t2, trap_w;   // harmonic trap
    double *R[2];                   // node positions by step parity, interleaved x, y
    double *fnode;                  // node forces at the current time (2n)
    int *origin;                    // patch origin by step parity: [parity][4] = unwrapped x, y
                                    // (node coordinates), then x mod nx, y mod ny
    float *fib;                     // spread force patch: 2 planes ps*ps
    float *vib;                     // fluid velocity patch: 2 planes ps*ps
    float *nw;                      // per node: the 4 x and 4 y kernel weights of its footprint
    int *nix;                       // per node: first footprint site (unwrapped x, y)
};

// fused kernel work item: columns [x0, x0+w), rows [y0, y0+l) of one simulation; full: the strip
// is the whole lattice width (x0 = 0, w = nx), its lanes' neighbours wrap within it
struct WorkItem {
    int sim, x0, y0, w, l, full, pad1, pad2;
};

// multi-pass kernels: one 256-site block of one simulation
struct SiteBlock {
    int sim, start;
};

}  // namespace lbk
