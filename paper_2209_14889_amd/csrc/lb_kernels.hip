// HIP kernels of liblb for gfx950 (MI355X).
//
//   k_ib_step     immersed-body update (App. A): node Heun step, node forces and force spreading
//                 in one launch, for a step with few patch tiles
//   k_ib_nodes, k_ib_spread   the same in two launches (nodes once per body, then the tiles)
//   k_fused       one pass per step over every lattice site: forces, BGK + Guo collide with pull
//                 streaming, velocity gradient, stiffness, Heun stress and polarization
//   k_mp_*        the same step as four simple site-parallel kernels (debug / reference path)
//   k_readout     observables at the current time
//   k_sums / k_sums_final, k_body_force   FP64 reductions
//
// The fused kernel walks a strip of columns down its rows like a pipeline.  Iteration j loads the
// polarization of row f = y0 - 4 + j and the stress of row f-1, forms the Ericksen stress at row
// f-1, collides row f-2, predicts row f-3 and corrects row f-4.  Every stage only needs rows that
// earlier stages or earlier iterations produced, so within a work item each value is computed
// once (the items overlap only by the pipeline's halo rows and columns) and row exchanges go
// through small LDS ring buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <hip/hip_fp16.h>

#include "lb_device.h"
#include "lb_launch.h"

namespace lbk {

// ------------------------------------------------------------------------------------------------
// immersed boundary
// ------------------------------------------------------------------------------------------------

// the four x (or y) weights phi(R - i), i = floor(R) - 1 .. floor(R) + 2, of the cosine kernel
// phi(r) = (1 + cos(pi r / 2)) / 4 (App. A).  With f = R - floor(R) in [0, 1) the four distances
// are 1 + f, f, f - 1, f - 2, whose cosines are -sin, cos, sin, -cos of pi f / 2: one sincos
// gives all four (the last weight is 0 at f = 0, where its site leaves the support |r| < 2).
// FP32 is enough for weights of values that are themselves FP32.
__device__ __forceinline__ void phi4(double R, int &i0, float w[4]) {
    const double fl = floor(R);
    i0 = (int)fl - 1;
    const float f = (float)(R - fl);
    float sn, cs;
    sincosf(1.57079632679f * f, &sn, &cs);
    w[0] = 0.25f * (1.0f - sn);
    w[1] = 0.25f * (1.0f + cs);
    w[2] = 0.25f * (1.0f + sn);
    w[3] = 0.25f * (1.0f - cs);
}

__device__ __forceinline__ double pull_factor(const BodyDev &B, double t) {
    if (B.width <= 0.0) return 1.0;
    return 1.0 / (1.0 + exp(-(t - B.t_on) / B.width)) - 1.0 / (1.0 + exp(-(t - B.t_off) / B.width));
}

// v at point R from a body's velocity patch V (side ps, origin ox, oy; the x plane, then the y
// plane); flags reads outside the patch
__device__ __forceinline__ void interp_patch(const float *V, int ps, int ox, int oy, double Rx, double Ry,
                                             double &vx, double &vy, bool &bad) {
    int ix, iy;
    float wx[4], wy[4];
    phi4(Rx, ix, wx);
    phi4(Ry, iy, wy);
    const size_t pp = (size_t)ps * ps;
    vx = 0.0;
    vy = 0.0;
    const int px0 = ix - ox, py0 = iy - oy;
    if (px0 < 0 || py0 < 0 || px0 + 3 >= ps || py0 + 3 >= ps) {
        bad = true;
        return;
    }
    for (int j = 0; j < 4; ++j) {
        double ax = 0.0, ay = 0.0;
        const size_t q = (size_t)(py0 + j) * ps + px0;
        for (int i = 0; i < 4; ++i) {
            ax += (double)wx[i] * (double)V[q + i];
            ay += (double)wx[i] * (double)V[pp + q + i];
        }
        vx += (double)wy[j] * ax;
        vy += (double)wy[j] * ay;
    }
}

// Heun step of one node through the velocity patch V: R + (v(R) + v(R + v(R))) / 2
__device__ __forceinline__ void heun_node(const float *V, int ps, int ox, int oy, double2 &R, bool &bad) {
    double v1x, v1y, v2x, v2y;
    interp_patch(V, ps, ox, oy, R.x, R.y, v1x, v1y, bad);
    interp_patch(V, ps, ox, oy, R.x + v1x, R.y + v1y, v2x, v2y, bad);
    R.x += 0.5 * (v1x + v2x);
    R.y += 0.5 * (v1y + v2y);
}

// derivative of cos(gamma_j) with respect to e1 = R_{j-1} - R_j (d1) and e2 = R_{j+1} - R_j (d2)
__device__ __forceinline__ void angle_grads(const double2 *R, int n, int j, double2 &d1, double2 &d2) {
    int jm = j == 0 ? n - 1 : j - 1, jp = j == n - 1 ? 0 : j + 1;
    double e1x = R[jm].x - R[j].x, e1y = R[jm].y - R[j].y;
    double e2x = R[jp].x - R[j].x, e2y = R[jp].y - R[j].y;
    double n1 = sqrt(e1x * e1x + e1y * e1y), n2 = sqrt(e2x * e2x + e2y * e2y);
    double in12 = 1.0 / (n1 * n2);
    double cg = (e1x * e2x + e1y * e2y) * in12;
    d1.x = e2x * in12 - cg * e1x / (n1 * n1);
    d1.y = e2y * in12 - cg * e1y / (n1 * n1);
    d2.x = e1x * in12 - cg * e2x / (n2 * n2);
    d2.y = e1y * in12 - cg * e2y / (n2 * n2);
}

// spring force k (l - l_eq) d/l on node i from the spring to node j (d = R_j - R_i)
__device__ __forceinline__ double2 spring_pull(const double2 *R, int i, int j, double k, double leq) {
    double dx = R[j].x - R[i].x, dy = R[j].y - R[i].y;
    double l = sqrt(dx * dx + dy * dy);
    double c = k * (l - leq) / l;
    return make_double2(c * dx, c * dy);
}

// -dU/dR_a for U = sum springs + sum bending (eqConst), plus the pull share
__device__ __forceinline__ double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// centre of mass of the n nodes in LDS, the same in every block: per-thread sums in node order,
// wave sums, then the four waves in a fixed order (256-thread blocks)
__device__ __forceinline__ double2 block_com(const double2 *sR, int n, double (*sC)[2]) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double cx = 0.0, cy = 0.0;
    for (int a = tid; a < n; a += 256) {
        cx += sR[a].x;
        cy += sR[a].y;
    }
    cx = wave_sum(cx);
    cy = wave_sum(cy);
    if (lane == 0) {
        sC[wv][0] = cx;
        sC[wv][1] = cy;
    }
    __syncthreads();
    return make_double2(((sC[0][0] + sC[1][0]) + (sC[2][0] + sC[3][0])) / n,
                        ((sC[0][1] + sC[1][1]) + (sC[2][1] + sC[3][1])) / n);
}

// each node's share k(t) (R_ext(t) - R_com) / n of the harmonic trap (App. A, eqUtrap): stiffness
// switched by logistics, trap moved by their integral (a smoothed constant-speed ramp)
__device__ __forceinline__ double2 trap_share(const BodyDev &B, double t, double2 com) {
    if (B.trap_k == 0.0) return make_double2(0.0, 0.0);
    const double w = B.trap_w, T = B.trap_t2 - B.trap_t1;
    const double u1 = (t - B.trap_t1) / w, u2 = (t - B.trap_t2) / w;
    const double k = B.trap_k * (1.0 / (1.0 + exp(-u1)) - 1.0 / (1.0 + exp(-u2)));
    auto sp = [](double x) { return x > 30.0 ? x + log1p(exp(-x)) : log1p(exp(x)); };
    const double rho = T > 0.0 ? (w / T) * (sp(u1) - sp(u2)) : 0.0;
    return make_double2(k * (B.trap_x0 + B.trap_dx * rho - com.x) / B.n, k * (B.trap_y0 + B.trap_dy * rho - com.y) / B.n);
}

__device__ __forceinline__ double2 node_force(const BodyDev &B, const double2 *R, int a, double pf, double2 trap) {
    const int n = B.n;
    int am = a == 0 ? n - 1 : a - 1, ap = a == n - 1 ? 0 : a + 1;
    double2 s1 = spring_pull(R, a, ap, B.k, B.leq);
    double2 s0 = spring_pull(R, a, am, B.k, B.leq);
    double2 d1a, d2a, d1m, d2m, d1p, d2p;
    angle_grads(R, n, a, d1a, d2a);
    angle_grads(R, n, am, d1m, d2m);
    angle_grads(R, n, ap, d1p, d2p);
    double fx = s1.x + s0.x + B.eps * ((d1a.x + d2a.x) - d2m.x - d1p.x) + pf * B.fx / n + trap.x;
    double fy = s1.y + s0.y + B.eps * ((d1a.y + d2a.y) - d2m.y - d1p.y) + pf * B.fy / n + trap.y;
    return make_double2(fx, fy);
}


// Two-launch body update for many bodies (each node advanced once): k_ib_nodes, then k_ib_spread.
// One block per body.  ADVANCE: move the nodes from R(t) to R(t+1) by Heun with the velocity patch
// written during step t (App. A: overdamped, no slip); otherwise take R[cur] as it is.  Then the
// node forces at the new positions with the pull at time *d_t, the new patch origin, and each
// node's footprint weights for the spreading kernel.
template <bool ADVANCE>
__global__ __launch_bounds__(256) void k_ib_nodes(const SimDev *__restrict__ sims, BodyDev *__restrict__ bodies,
                                                  int cur, const int *__restrict__ d_t, int *__restrict__ d_status) {
    __shared__ double2 sR[kMaxNodes];
    __shared__ double sRed[4][4];
    __shared__ double sC[4][2];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const BodyDev &B = bodies[blockIdx.x];
    const SimDev &S = sims[B.sim];
    const int n = B.n;
    const int dst = ADVANCE ? (cur ^ 1) : cur;
    bool bad = false;
    bool wall = false;   // a node's kernel footprint reaches a wall

    const double2 *Rc = reinterpret_cast<const double2 *>(B.R[cur]);
    int ox = 0, oy = 0;
    if (ADVANCE) {
        ox = B.origin[4 * cur];
        oy = B.origin[4 * cur + 1];
    }
    for (int a = tid; a < n; a += 256) {
        double2 R = Rc[a];
        if (ADVANCE) heun_node(B.vib, B.ps, ox, oy, R, bad);
        sR[a] = R;
    }
    __syncthreads();

    const double pf = pull_factor(B, (double)d_t[0]);
    const double2 trap = trap_share(B, (double)d_t[0], block_com(sR, n, sC));
    double2 *Fn = reinterpret_cast<double2 *>(B.fnode);
    double2 *Rd = reinterpret_cast<double2 *>(B.R[dst]);
    double mnx = 1e300, mny = 1e300, mxx = -1e300, mxy = -1e300;
    for (int a = tid; a < n; a += 256) {
        const double2 R = sR[a];
        Fn[a] = node_force(B, sR, a, pf, trap);
        if (ADVANCE) Rd[a] = R;
        int ix, iy;
        float wx[4], wy[4];
        phi4(R.x, ix, wx);
        phi4(R.y, iy, wy);
        if ((S.walls && (iy < 1 || iy + 4 >= S.ny)) || (S.walls == 2 && (ix < 1 || ix + 4 >= S.nx)))
            wall = true;   // one site of margin for the predicted position
        B.nix[2 * a] = ix;
        B.nix[2 * a + 1] = iy;
        float4 *w = reinterpret_cast<float4 *>(B.nw) + 2 * a;
        w[0] = make_float4(wx[0], wx[1], wx[2], wx[3]);
        w[1] = make_float4(wy[0], wy[1], wy[2], wy[3]);
        mnx = fmin(mnx, R.x);
        mny = fmin(mny, R.y);
        mxx = fmax(mxx, R.x);
        mxy = fmax(mxy, R.y);
    }
    mnx = wave_min(mnx);
    mny = wave_min(mny);
    mxx = wave_max(mxx);
    mxy = wave_max(mxy);
    if (lane == 0) {
        sRed[wv][0] = mnx;
        sRed[wv][1] = mny;
        sRed[wv][2] = mxx;
        sRed[wv][3] = mxy;
    }
    __syncthreads();
    if (tid == 0) {
        mnx = fmin(fmin(sRed[0][0], sRed[1][0]), fmin(sRed[2][0], sRed[3][0]));
        mny = fmin(fmin(sRed[0][1], sRed[1][1]), fmin(sRed[2][1], sRed[3][1]));
        mxx = fmax(fmax(sRed[0][2], sRed[1][2]), fmax(sRed[2][2], sRed[3][2]));
        mxy = fmax(fmax(sRed[0][3], sRed[1][3]), fmax(sRed[2][3], sRed[3][3]));
        // patch: 3 sites of margin below the lowest node cover the kernel support (2) plus one
        // site of node motion; the same margin above is checked against the patch side
        const int nox = (int)floor(mnx) - 3, noy = (int)floor(mny) - 3;
        if ((int)floor(mxx) + 3 - nox >= B.ps || (int)floor(mxy) + 3 - noy >= B.ps) bad = true;
        B.origin[4 * dst] = nox;
        B.origin[4 * dst + 1] = noy;
        B.origin[4 * dst + 2] = wrapi(nox, S.nx);
        B.origin[4 * dst + 3] = wrapi(noy, S.ny);
    }
    if (bad) atomicOr(d_status, kStatusPatch);
    if (wall) atomicOr(d_status, kStatusWall);
}

// f_IB at tile site (lx, ly) = sum over the listed nodes, in list (node) order, of
// f_a phi(x) phi(y), from each node's 4x4 footprint origin o (tile coordinates) and its
// separable weights.  The LDS reads of four nodes are issued before any of them is used, so
// each group of four costs one LDS round trip instead of two per node.
__device__ __forceinline__ void gather_one(int lx, int ly, int2 o, float4 wxv, float4 wyv, double2 f, double &fx,
                                           double &fy) {
    const int i = lx - o.x, jj = ly - o.y;
    if ((unsigned)i < 4u && (unsigned)jj < 4u) {
        const float wxs = i == 0 ? wxv.x : i == 1 ? wxv.y : i == 2 ? wxv.z : wxv.w;
        const float wys = jj == 0 ? wyv.x : jj == 1 ? wyv.y : jj == 2 ? wyv.z : wyv.w;
        const double w = (double)wxs * (double)wys;
        fx += f.x * w;
        fy += f.y * w;
    }
}
__device__ __forceinline__ void gather_site(const int2 *sI, const float4 (*sW)[2], const double2 *sF, int cnt, int lx,
                                            int ly, double &fx, double &fy) {
    int q = 0;
    for (; q + 4 <= cnt; q += 4) {
        int2 o[4];
        float4 wx[4], wy[4];
        double2 f[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            o[u] = sI[q + u];
            wx[u] = sW[q + u][0];
            wy[u] = sW[q + u][1];
            f[u] = sF[q + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) gather_one(lx, ly, o[u], wx[u], wy[u], f[u], fx, fy);
    }
    for (; q < cnt; ++q) gather_one(lx, ly, sI[q], sW[q][0], sW[q][1], sF[q], fx, fy);
}

// One block per (body, 16x16 tile of its patch): f_IB(r) = sum_a f_a phi phi (App. A) as a gather
// over the nodes whose 4x4 footprint reaches the tile, summed in node order (deterministic).
__global__ __launch_bounds__(256) void k_ib_spread(const BodyDev *__restrict__ bodies, const int2 *__restrict__ blk,
                                                   int dst, int *__restrict__ d_status) {
    __shared__ int sA[kMaxCand];
    __shared__ int2 sI[kMaxCand];
    __shared__ float4 sW[kMaxCand][2];
    __shared__ double2 sF[kMaxCand];
    __shared__ int sCnt[4];
    __shared__ int sTot;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int2 bt = blk[blockIdx.x];
    const BodyDev &B = bodies[bt.x];
    const int n = B.n;
    const int tx = bt.y % B.nside, ty = bt.y / B.nside;
    const int X0 = B.origin[4 * dst] + tx * kPatchTile, Y0 = B.origin[4 * dst + 1] + ty * kPatchTile;
    if (tid == 0) sTot = 0;
    __syncthreads();
    bool bad = false;
    for (int base = 0; base < n; base += 256) {
        const int a = base + tid;
        bool flag = false;
        int ix = 0, iy = 0;
        if (a < n) {
            ix = B.nix[2 * a];
            iy = B.nix[2 * a + 1];
            flag = ix > X0 - 4 && ix < X0 + kPatchTile && iy > Y0 - 4 && iy < Y0 + kPatchTile;
        }
        const unsigned long long m = __ballot(flag);
        const int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) sCnt[wv] = __popcll(m);
        __syncthreads();
        int off = sTot;
        for (int w = 0; w < wv; ++w) off += sCnt[w];
        if (flag) {
            const int q = off + pre;
            if (q < kMaxCand) {
                sA[q] = a;
                sI[q] = make_int2(ix - X0, iy - Y0);
                const float4 *w = reinterpret_cast<const float4 *>(B.nw) + 2 * a;
                sW[q][0] = w[0];
                sW[q][1] = w[1];
                sF[q] = reinterpret_cast<const double2 *>(B.fnode)[a];
            } else {
                bad = true;
            }
        }
        __syncthreads();
        if (tid == 0) sTot += sCnt[0] + sCnt[1] + sCnt[2] + sCnt[3];
        __syncthreads();
    }
    const int cnt = min(sTot, kMaxCand);
    const int lx = tid % kPatchTile, ly = tid / kPatchTile;
    const int px = tx * kPatchTile + lx, py = ty * kPatchTile + ly;
    if (px < B.ps && py < B.ps) {
        double fx = 0.0, fy = 0.0;
        gather_site(sI, sW, sF, cnt, lx, ly, fx, fy);
        const unsigned i = (unsigned)(py * B.ps + px);
        B.fib[i] = (float)fx;
        B.fib[(unsigned)(B.ps * B.ps) + i] = (float)fy;
    }
    if (bad) atomicOr(d_status, kStatusPatch);
}

// Body update and force spreading in one launch, one 256-thread block per (body, 16x16 tile of
// its patch).  Every block of a body repeats the node update (a few hundred nodes):
//  ADVANCE: move the nodes from R(t) to R(t+1) by Heun with the velocity patch written during
//  step t (App. A: overdamped, no slip); otherwise take R[cur] as it is;
//  the patch origin for the new positions (3 sites of margin around the nodes), found in the same
//  pass as the centre of mass;
//  every node's force at the new positions with the pull at time *d_t (once, each by the thread
//  that lists the node), and of those the nodes whose 4x4 footprint reaches the tile gathered onto
//  the tile's sites in node order (deterministic): f_IB(r) = sum_a f_a phi phi (App. A).
// Tile 0 of each body publishes the new positions, all node forces and the origin; the other
// blocks only read the current-parity buffers, so blocks never wait on each other.
template <bool ADVANCE>
__global__ __launch_bounds__(256) void k_ib_step(const SimDev *__restrict__ sims, BodyDev *__restrict__ bodies,
                                                 const int2 *__restrict__ blk, int cur, const int *__restrict__ d_t,
                                                 int *__restrict__ d_status) {
    __shared__ double2 sR[kMaxNodes];
    __shared__ double sRed[4][4];
    __shared__ int2 sI[kMaxCand];
    __shared__ float4 sW[kMaxCand][2];
    __shared__ double2 sF[kMaxCand];
    __shared__ double2 sFall[kMaxNodes];   // every node's force (each thread's own nodes)
    __shared__ int sCnt[4];
    __shared__ double sC[4][2];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int2 bt = blk[blockIdx.x];
    BodyDev &B = bodies[bt.x];
    const SimDev &S = sims[B.sim];
    const int n = B.n;
    const int dst = ADVANCE ? (cur ^ 1) : cur;
    const bool lead = bt.y == 0;
    bool bad = false;        // node outside its patch (every block finds the same; tile 0 reports)
    bool overflow = false;   // more footprints reach this tile than it can list
    bool wall = false;       // a node's kernel footprint reaches a wall

    const double2 *Rc = reinterpret_cast<const double2 *>(B.R[cur]);
    int ox = 0, oy = 0;
    if (ADVANCE) {
        ox = B.origin[4 * cur];
        oy = B.origin[4 * cur + 1];
    }
    // one pass for the extent and the centre of mass (the sums in block_com's order)
    double mnx = 1e300, mny = 1e300, mxx = -1e300, mxy = -1e300, cx = 0.0, cy = 0.0;
    for (int a = tid; a < n; a += 256) {
        double2 R = Rc[a];
        if (ADVANCE) heun_node(B.vib, B.ps, ox, oy, R, bad);
        sR[a] = R;
        mnx = fmin(mnx, R.x);
        mny = fmin(mny, R.y);
        mxx = fmax(mxx, R.x);
        mxy = fmax(mxy, R.y);
        cx += R.x;
        cy += R.y;
    }
    mnx = wave_min(mnx);
    mny = wave_min(mny);
    mxx = wave_max(mxx);
    mxy = wave_max(mxy);
    cx = wave_sum(cx);
    cy = wave_sum(cy);
    if (lane == 0) {
        sRed[wv][0] = mnx;
        sRed[wv][1] = mny;
        sRed[wv][2] = mxx;
        sRed[wv][3] = mxy;
        sC[wv][0] = cx;
        sC[wv][1] = cy;
    }
    __syncthreads();
    const double2 com = make_double2(((sC[0][0] + sC[1][0]) + (sC[2][0] + sC[3][0])) / n,
                                     ((sC[0][1] + sC[1][1]) + (sC[2][1] + sC[3][1])) / n);
    mnx = fmin(fmin(sRed[0][0], sRed[1][0]), fmin(sRed[2][0], sRed[3][0]));
    mny = fmin(fmin(sRed[0][1], sRed[1][1]), fmin(sRed[2][1], sRed[3][1]));
    mxx = fmax(fmax(sRed[0][2], sRed[1][2]), fmax(sRed[2][2], sRed[3][2]));
    mxy = fmax(fmax(sRed[0][3], sRed[1][3]), fmax(sRed[2][3], sRed[3][3]));
    // patch: 3 sites of margin below the lowest node cover the kernel support (2) plus one site of
    // node motion; the same margin above is checked against the patch side
    const int nox = (int)floor(mnx) - 3, noy = (int)floor(mny) - 3;
    if ((int)floor(mxx) + 3 - nox >= B.ps || (int)floor(mxy) + 3 - noy >= B.ps) bad = true;

    const double pf = pull_factor(B, (double)d_t[0]);
    const double2 trap = trap_share(B, (double)d_t[0], com);
    // every node's force once, by the thread that lists the node below (so no barrier)
    for (int a = tid; a < n; a += 256) sFall[a] = node_force(B, sR, a, pf, trap);
    if (lead) {
        double2 *Fn = reinterpret_cast<double2 *>(B.fnode);
        double2 *Rd = reinterpret_cast<double2 *>(B.R[dst]);
        for (int a = tid; a < n; a += 256) {
            Fn[a] = sFall[a];
            if (ADVANCE) Rd[a] = sR[a];
        }
        if (tid == 0) {
            B.origin[4 * dst] = nox;
            B.origin[4 * dst + 1] = noy;
            B.origin[4 * dst + 2] = wrapi(nox, S.nx);
            B.origin[4 * dst + 3] = wrapi(noy, S.ny);
        }
    }

    // nodes whose footprint reaches this tile, compacted in node order
    const int tx = bt.y % B.nside, ty = bt.y / B.nside;
    const int X0 = nox + tx * kPatchTile, Y0 = noy + ty * kPatchTile;
    int tot = 0;
    for (int base = 0; base < n; base += 256) {
        const int a = base + tid;
        bool flag = false;
        int ix = 0, iy = 0;
        float wx[4], wy[4];
        if (a < n) {
            const double2 R = sR[a];
            phi4(R.x, ix, wx);
            phi4(R.y, iy, wy);
            if ((S.walls && (iy < 1 || iy + 4 >= S.ny)) || (S.walls == 2 && (ix < 1 || ix + 4 >= S.nx)))
            wall = true;   // one site of margin for the predicted position
            flag = ix > X0 - 4 && ix < X0 + kPatchTile && iy > Y0 - 4 && iy < Y0 + kPatchTile;
        }
        const unsigned long long m = __ballot(flag);
        const int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) sCnt[wv] = __popcll(m);
        __syncthreads();
        int off = tot;
        for (int w = 0; w < wv; ++w) off += sCnt[w];
        if (flag) {
            const int q = off + pre;
            if (q < kMaxCand) {
                sI[q] = make_int2(ix - X0, iy - Y0);
                sW[q][0] = make_float4(wx[0], wx[1], wx[2], wx[3]);
                sW[q][1] = make_float4(wy[0], wy[1], wy[2], wy[3]);
                sF[q] = sFall[a];
            } else {
                overflow = true;
            }
        }
        tot += sCnt[0] + sCnt[1] + sCnt[2] + sCnt[3];
        __syncthreads();
    }
    const int cnt = min(tot, kMaxCand);
    const int lx = tid % kPatchTile, ly = tid / kPatchTile;
    const int px = tx * kPatchTile + lx, py = ty * kPatchTile + ly;
    if (px < B.ps && py < B.ps) {
        double fx = 0.0, fy = 0.0;
        gather_site(sI, sW, sF, cnt, lx, ly, fx, fy);
        const unsigned i = (unsigned)(py * B.ps + px);
        B.fib[i] = (float)fx;
        B.fib[(unsigned)(B.ps * B.ps) + i] = (float)fy;
    }
    if ((bad && lead) || overflow) atomicOr(d_status, kStatusPatch);
    if (wall && lead) atomicOr(d_status, kStatusWall);
}

// ------------------------------------------------------------------------------------------------
// fused single-pass step
// ------------------------------------------------------------------------------------------------

// blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous run of work items so
// neighbouring strips and segments share that XCD's L2
__device__ __forceinline__ int xcd_remap(int v, int n) {
    int q = n >> 3, r = n & 7;
    int x = v & 7, k = v >> 3;
    return x * q + min(x, r) + k;
}

__device__ __forceinline__ void inc_row(unsigned &r, unsigned ny) { r = (r + 1u == ny) ? 0u : r + 1u; }

// POL = false: every simulation of the launch has P = 0, which the dynamics keep exactly (the
// polarization right-hand side is proportional to P), so the Ericksen stress vanishes and C~ is
// its isotropic value: the scalar model of Sec. II B.  That variant skips all P work.
template <int T, typename HT, bool WALLS, bool POL>
__global__ __launch_bounds__(T, (WALLS || !std::is_same<HT, __half>::value) ? 3 : 4) void k_fused(const SimDev *__restrict__ sims, const BodyDev *__restrict__ bodies,
                                             const WorkItem *__restrict__ items, int n_items, int cur,
                                             int *__restrict__ d_t, int cus) {
    // row-exchange rings; values a thread needs only from its own column one row below live in
    // registers (the "carried" row of the previous iteration)
    typedef typename PolOf<HT>::T PT;   // polarization storage: FP32 offsets with FP16 populations, else FP64
    constexpr int TP = POL ? T : 1;   // the P rings exist only in the variant with P
    __shared__ PT rP[4][2][TP];       // polarization, rows f-3 .. f
    __shared__ float rS[3][3][T];     // stress rows f-3 .. f-1
    __shared__ float rE[2][2][TP];    // Ericksen xx and yx, rows f-2 .. f-1
    __shared__ float rV[2][2][T];     // half-velocity rows f-3 .. f-2
    __shared__ float rQs[2][3][T];    // predicted stress rows f-4 .. f-3
    __shared__ PT rQp[2][2][TP];      // predicted polarization, rows f-4 .. f-3
    __shared__ float4 sTab[2 * kStiffSeg];     // stiffness cubics of the item's simulation
    __shared__ ItemBody sIB[kItemBodies];      // bodies whose patches touch the item
    __shared__ int sNB;                        // their number, -1 if more than kItemBodies
    const int tid = threadIdx.x;
    const int nxt = cur ^ 1;
    if (blockIdx.x == 0 && tid == 0) d_t[0] = d_t[0] + 1;   // the body update after this step uses t+1

    for (int vi = blockIdx.x; vi < n_items; vi += gridDim.x) {
        __syncthreads();   // the previous item's last stages have read the item tables below
        const WorkItem wi = items[xcd_remap(vi, n_items)];
        const SimDev &S = sims[wi.sim];
        const unsigned nx = (unsigned)S.nx, ny = (unsigned)S.ny;
        const unsigned N = nx * ny;
        const HT *__restrict__ hin = reinterpret_cast<const HT *>(S.h[cur]);
        HT *__restrict__ hout = reinterpret_cast<HT *>(S.h[nxt]);
        const float *__restrict__ sgi = S.sig[cur];
        float *__restrict__ sgo = S.sig[nxt];
        const PT *__restrict__ Pi = static_cast<const PT *>(S.P[cur]);
        PT *__restrict__ Po = static_cast<PT *>(S.P[nxt]);
        // A strip of w columns takes lanes 0 .. w+7: 4 halo columns on each side, recomputed by
        // the neighbouring strip.  A lattice no wider than the work-group is one full-width strip
        // (wi.full): lane = column, no halo lanes, and a lane's east and west neighbours wrap
        // around within the strip.  Lanes beyond the strip idle (whole waves skip every stage).
        const bool full = wi.full != 0;
        const int lanes = full ? wi.w : wi.w + 2 * kHalo;
        const bool live = tid < lanes;
        const int c = full ? (live ? tid : 0) : wi.x0 - kHalo + tid;
        const unsigned x = (unsigned)wrapi(c, (int)nx), xm = (unsigned)wrapi(c - 1, (int)nx),
                       xp = (unsigned)wrapi(c + 1, (int)nx);
        const int wcol = wi.w;
        const bool colB = full ? live : tid >= 1 && tid < wcol + 7;
        const bool colC = full ? live : tid >= 2 && tid < wcol + 6;
        const bool colD = full ? live : tid >= 3 && tid < wcol + 5;
        const bool colE = full ? live : tid >= 4 && tid < wcol + 4;
        const float is = S.inv_scale, sc = S.scale;

        // per-item constants: the stiffness cubics, and the bodies whose patches reach the rows
        // y0-2 .. y0+l+1 and columns x0-4 .. x0+w+3 this item touches (wave 0 holds every body:
        // at most kMaxBodies = 64 per simulation)
        for (int q = tid; q < 2 * kStiffSeg; q += T) sTab[q] = reinterpret_cast<const float4 *>(S.tab)[q];
        if (tid < 64) {
            bool hit = false;
            ItemBody ib{0, 0, 0, 0, nullptr, nullptr};
            if (tid < S.nb) {
                const BodyDev &B = bodies[S.b0 + tid];
                ib.ox = gptr(B.origin)[4 * cur + 2];
                ib.oy = gptr(B.origin)[4 * cur + 3];
                ib.ps = B.ps;
                ib.fib = B.fib;
                ib.vib = B.vib;
                hit = ring_overlap(ib.ox, ib.ps, full ? 0 : wrapi(wi.x0 - kHalo, (int)nx), lanes, (int)nx) &&
                      ring_overlap(ib.oy, ib.ps, wrapi(wi.y0 - 2, (int)ny), wi.l + 4, (int)ny);
            }
            const unsigned long long m = __ballot(hit);
            const int cnt = __popcll(m);
            if (hit) {
                const int k = __popcll(m & ((1ull << tid) - 1ull));
                if (k < kItemBodies) sIB[k] = ib;
            }
            if (tid == 0) sNB = cnt <= kItemBodies ? cnt : -1;
        }

        // wrapped row indices relative to the front row f of the current iteration
        // (the rows of iteration 2, where the pipeline starts: f = f0 + 2)
        const int f0 = wi.y0 - 4, f2 = f0 + 2;
        unsigned rp1 = (unsigned)wrapi(f2 + 1, (int)ny), r0 = (unsigned)wrapi(f2, (int)ny);
        unsigned rm1 = (unsigned)wrapi(f2 - 1, (int)ny), rm2 = (unsigned)wrapi(f2 - 2, (int)ny);
        unsigned rm3 = (unsigned)wrapi(f2 - 3, (int)ny), rm4 = (unsigned)wrapi(f2 - 4, (int)ny);
        // walls: the rows next to them, whose neighbour beyond is a ghost
        const bool walls = WALLS && S.walls != 0;   // the periodic variant has no wall code
        const unsigned ytop = ny - 1u;
        // closed box: this lane's column is next to the west / east wall
        const bool xw = WALLS && S.walls == 2 && x == 0u, xe = WALLS && S.walls == 2 && x == nx - 1u;
        // the lanes holding the east and west neighbours (the lane itself beyond a wall: mirror
        // ghosts; wrapped around a full-width strip)
        const int te = xe ? tid : (full && tid + 1 == lanes ? 0 : tid + 1);
        const int tw = xw ? tid : (full && tid == 0 ? lanes - 1 : tid - 1);
        // this lane's column and its neighbours as byte offsets within a row of populations (HT)
        // and of the 4-byte stress and polarization planes; the state arrays as buffers
        const unsigned HB = (unsigned)sizeof(HT);
        const unsigned bh = x * HB, bhm = xm * HB, bhp = xp * HB;
        const unsigned b4 = x * 4u, bP = x * (unsigned)sizeof(PT);
        const __amdgpu_buffer_rsrc_t rHi = state_rsrc(hin), rHo = state_rsrc(hout), rSi = state_rsrc(sgi),
                                     rSo = state_rsrc(sgo), rPi = state_rsrc(Pi), rPo = state_rsrc(Po);

        // Loads for the next iteration, issued one iteration ahead.  Every lane loads (all
        // indices are wrapped into the lattice); lanes outside a stage's columns never use them.
        struct Pre {
            PT P0, P1;                     // P(f+1)
            float S0, S1, S2;              // sigma(f)
            typename Pop<HT>::Raw H[9];    // populations pulled into row f-1
        };
        // Values of this column handed from one iteration to the next: stage D's centre row
        // (the corrector's frozen inputs and the next predictor's south neighbours) and stage E's
        // predicted centre (the next corrector's south neighbour).
        struct Carry {
            float hx, hy, s0, s1, s2;      // hx, hy: half the velocity
            PT p0, p1;
            Grad g;
            Stiff k;
            float q0, q1, q2;
            PT qp0, qp1;
        };
        Pre preA, preB;
        Carry carA, carB;
        // Row iterations 0 and 1 would only commit P rows f0 and f0+1 (their stress rows f0-1 and
        // f0 are read by no stage), so the pipeline starts at iteration 2: those two P rows go
        // into the ring here, with one wait, and preA takes iteration 2's rows.
        if (live) {
            const unsigned rP0 = r0 * nx * (unsigned)sizeof(PT), NP = N * (unsigned)sizeof(PT);
            const unsigned rS0 = rm1 * nx * 4u, N4 = N * 4u;
            if (POL) {
                const unsigned rF0 = rm2 * nx * (unsigned)sizeof(PT), rF1 = rm1 * nx * (unsigned)sizeof(PT);
                PT f00, f01, f10, f11;
                buf_ld(rPi, bP, rF0, f00);
                buf_ld(rPi, bP, NP + rF0, f01);
                buf_ld(rPi, bP, rF1, f10);
                buf_ld(rPi, bP, NP + rF1, f11);
                buf_ld(rPi, bP, rP0, preA.P0);
                buf_ld(rPi, bP, NP + rP0, preA.P1);
                rP[0][0][tid] = f00;
                rP[0][1][tid] = f01;
                rP[1][0][tid] = f10;
                rP[1][1][tid] = f11;
            }
            preA.S0 = buf_ldf(rSi, b4, rS0);
            preA.S1 = buf_ldf(rSi, b4, N4 + rS0);
            preA.S2 = buf_ldf(rSi, b4, 2u * N4 + rS0);
        }
        // Ericksen xy, yy of this column at rows f-1, f-2, f-3
        float exy1 = 0.f, eyy1 = 0.f, exy2 = 0.f, eyy2 = 0.f, exy3 = 0.f, eyy3 = 0.f;

        __syncthreads();
        const int nib = sNB;
        const int niter = wi.l + 8;

        // one row iteration j; pin/cin were filled by iteration j-1, pout/cout are for j+1
        auto iterate = [&](const int j, const Pre &pin, Pre &pout, const Carry &cin, Carry &cout) {
            const int a0 = j & 3, a1 = (j + 3) & 3, a2 = (j + 2) & 3, a3 = (j + 1) & 3;   // P rows f .. f-3
            const int b1 = (j + 59) % 3, b2 = (j + 58) % 3, b3 = (j + 57) % 3;           // stress rows f-1 .. f-3
            const int o1 = (j + 1) & 1, o0 = j & 1;   // rows f-1 / f-3 (odd lag) and f-2 / f-4 (even lag)

            // One barrier per iteration.  Every value a stage reads from another lane was written
            // in an earlier iteration (stage B reads P rows written by A one or more iterations
            // ago, C the Ericksen row B wrote last iteration, D the velocity row C wrote last
            // iteration, E the predictor row D wrote last iteration); what a stage reads from the
            // current iteration is its own column, written by its own lane.  Every slot written
            // here last held a row that an earlier iteration read.  So one barrier between
            // consecutive iterations orders all of it.
            __syncthreads();

            // ---- stage A: commit P(f), sigma(f-1); take this iteration's populations
            if (POL) {
                rP[a0][0][tid] = pin.P0;
                rP[a0][1][tid] = pin.P1;
            }
            rS[b1][0][tid] = pin.S0;
            rS[b1][1][tid] = pin.S1;
            rS[b1][2][tid] = pin.S2;
            float d[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) d[q] = Pop<HT>::cvt_stored(pin.H[q]);   // times the storage scale
            // prefetch for iteration j+1: P(f+1), sigma(f), and the populations pulled into row
            // f-1: h_n(x, r) = h*_n(x - c_n, r - c_n) from rows f-2, f-1, f
            if (live && j + 1 < niter) {
                const unsigned rP1 = rp1 * nx * (unsigned)sizeof(PT), NP = N * (unsigned)sizeof(PT);
                const unsigned rS1 = r0 * nx * 4u, N4 = N * 4u;
                if (POL) {
                    buf_ld(rPi, bP, rP1, pout.P0);
                    buf_ld(rPi, bP, NP + rP1, pout.P1);
                }
                pout.S0 = buf_ldf(rSi, b4, rS1);
                pout.S1 = buf_ldf(rSi, b4, N4 + rS1);
                pout.S2 = buf_ldf(rSi, b4, 2u * N4 + rS1);
                if (!WALLS && j + 1 >= 4) {
                    // periodic: plane and row in the scalar offset, the column in the lane offset
                    const unsigned NH = N * HB, yc = rm1 * nx * HB, ym = rm2 * nx * HB, yp = r0 * nx * HB;
                    pout.H[0] = Pop<HT>::ld_buf(rHi, bh, yc);
                    pout.H[1] = Pop<HT>::ld_buf(rHi, bhm, NH + yc);
                    pout.H[2] = Pop<HT>::ld_buf(rHi, bh, 2u * NH + ym);
                    pout.H[3] = Pop<HT>::ld_buf(rHi, bhp, 3u * NH + yc);
                    pout.H[4] = Pop<HT>::ld_buf(rHi, bh, 4u * NH + yp);
                    pout.H[5] = Pop<HT>::ld_buf(rHi, bhm, 5u * NH + ym);
                    pout.H[6] = Pop<HT>::ld_buf(rHi, bhp, 6u * NH + ym);
                    pout.H[7] = Pop<HT>::ld_buf(rHi, bhp, 7u * NH + yp);
                    pout.H[8] = Pop<HT>::ld_buf(rHi, bhm, 8u * NH + yp);
                } else if (WALLS && j + 1 >= 4) {
                    const unsigned yc = rm1 * nx, ym = rm2 * nx, yp = r0 * nx;
                    // halfway bounce-back: what would come from beyond a wall is the opposite
                    // direction's post-collision value at the same site
                    const bool blo = walls && rm1 == 0u, bhi = walls && rm1 == ytop;
                    const unsigned own = yc + x;
                    pout.H[0] = Pop<HT>::ld_raw(hin, own);
                    pout.H[1] = Pop<HT>::ld_raw(hin, xw ? 3u * N + own : N + yc + xm);
                    pout.H[2] = Pop<HT>::ld_raw(hin, blo ? 4u * N + own : 2u * N + ym + x);
                    pout.H[3] = Pop<HT>::ld_raw(hin, xe ? N + own : 3u * N + yc + xp);
                    pout.H[4] = Pop<HT>::ld_raw(hin, bhi ? 2u * N + own : 4u * N + yp + x);
                    pout.H[5] = Pop<HT>::ld_raw(hin, blo || xw ? 7u * N + own : 5u * N + ym + xm);
                    pout.H[6] = Pop<HT>::ld_raw(hin, blo || xe ? 8u * N + own : 6u * N + ym + xp);
                    pout.H[7] = Pop<HT>::ld_raw(hin, bhi || xe ? 5u * N + own : 7u * N + yp + xp);
                    pout.H[8] = Pop<HT>::ld_raw(hin, bhi || xw ? 6u * N + own : 8u * N + yp + xm);
                }
            }

            // ---- stage B: Ericksen stress at row f-1
            exy3 = exy2;
            eyy3 = eyy2;
            exy2 = exy1;
            eyy2 = eyy1;
            if (POL && j >= 2 && colB) {
                const int an = walls && rm1 == ytop ? a1 : a0, as = walls && rm1 == 0u ? a1 : a2;
                PT Pc[2] = {rP[a1][0][tid], rP[a1][1][tid]};
                PT Pe[2] = {rP[a1][0][te], rP[a1][1][te]};
                PT Pw[2] = {rP[a1][0][tw], rP[a1][1][tw]};
                PT Pn[2] = {rP[an][0][tid], rP[an][1][tid]};
                PT Ps[2] = {rP[as][0][tid], rP[as][1][tid]};
                float E[4];
                ericksen(S, Pc, Pe, Pw, Pn, Ps, E);
                rE[o1][0][tid] = E[0];
                rE[o1][1][tid] = E[2];
                exy1 = E[1];
                eyy1 = E[3];
            }

            // ---- stage C: force, moments, collision at row f-2
            if (j >= 4 && colC) {
                const bool clo = walls && rm2 == 0u, chi = walls && rm2 == ytop;
                const int bn = chi ? b2 : b1, bs = clo ? b2 : b3;
                // twice the divergence of the stresses (central differences), halved once
                float fx = (rS[b2][0][te] - rS[b2][0][tw]) + (rS[bn][2][tid] - rS[bs][2][tid]);
                float fy = (rS[b2][2][te] - rS[b2][2][tw]) + (rS[bn][1][tid] - rS[bs][1][tid]);
                if (POL && S.ericksen) {
                    const float exn = chi ? exy2 : exy1, exs = clo ? exy2 : exy3;
                    const float eyn = chi ? eyy2 : eyy1, eys = clo ? eyy2 : eyy3;
                    fx += (rE[o0][0][te] - rE[o0][0][tw]) + (exn - exs);
                    fy += (rE[o0][1][te] - rE[o0][1][tw]) + (eyn - eys);
                }
                float Fx = fmaf(0.5f, fx, S.gx), Fy = fmaf(0.5f, fy, S.gy);
                if (nib > 0)
                    ib_force_list(sIB, nib, (int)nx, (int)ny, (int)x, (int)rm2, Fx, Fy);
                else if (nib < 0)
                    ib_force(S, bodies, cur, (int)x, (int)rm2, Fx, Fy);
                float drho, ux, uy;
                collide_t<Pop<HT>::kScaled>(d, Fx, Fy, S.omega, S.guo, sc, is, drho, ux, uy);
                rV[o0][0][tid] = 0.5f * ux;   // the gradient and advection stages take v / 2
                rV[o0][1][tid] = 0.5f * uy;
                const int r = wi.y0 + j - 6;   // = f - 2
                if (colE && r >= wi.y0 && r < wi.y0 + wi.l) {
                    const unsigned o = rm2 * nx * HB, NH = N * HB;
#pragma unroll
                    for (int q = 0; q < 9; ++q) Pop<HT>::st_buf(rHo, bh, (unsigned)q * NH + o, d[q]);
                    if (nib > 0)
                        ib_store_v_list(sIB, nib, (int)nx, (int)ny, (int)x, (int)rm2, ux, uy);
                    else if (nib < 0)
                        ib_store_v(S, bodies, cur, (int)x, (int)rm2, ux, uy);
                }
            }

            // ---- stage D: predictor at row f-3 (from j = 5 only the carried centre values)
            if (j >= 5 && colD) {
                cout.hx = rV[o1][0][tid];
                cout.hy = rV[o1][1][tid];
                PT Pc[2] = {POL ? rP[a3][0][tid] : (PT)0, POL ? rP[a3][1][tid] : (PT)0};
                float X[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) X[q] = rS[b3][q][tid];
                if (j >= 6) {
                    // walls: mirror ghosts for sigma and P, no-slip (negated) ghosts for v
                    const bool dlo = walls && rm3 == 0u, dhi = walls && rm3 == ytop;
                    const float vxn = dhi ? -cout.hx : rV[o0][0][tid], vyn = dhi ? -cout.hy : rV[o0][1][tid];
                    const float vxs = dlo ? -cout.hx : cin.hx, vys = dlo ? -cout.hy : cin.hy;
                    const float sxe = xe ? -1.0f : 1.0f, sxw = xw ? -1.0f : 1.0f;   // no-slip ghosts
                    cout.g = grad_v(sxe * rV[o1][0][te], sxw * rV[o1][0][tw], vxn, vxs,
                                    sxe * rV[o1][1][te], sxw * rV[o1][1][tw], vyn, vys);
                    // without P: the isotropic stiffness (all anisotropic parts vanish at P = 0)
                    cout.k = POL ? stiffness(S, sTab, (float)((PT)S.pref[0] + Pc[0]), (float)((PT)S.pref[1] + Pc[1]))
                                 : Stiff{0.f, 0.f, 0.f, 0.f};
                    float Xe[3], Xw[3], Xn[3], Rs[3];
                    const int bn = dhi ? b3 : b2;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        Xe[q] = rS[b3][q][te];
                        Xw[q] = rS[b3][q][tw];
                        Xn[q] = rS[bn][q][tid];
                    }
                    const float Xs[3] = {dlo ? X[0] : cin.s0, dlo ? X[1] : cin.s1, dlo ? X[2] : cin.s2};
                    rhs_sigma(S, cout.k, cout.g, cout.hx, cout.hy, X, Xe, Xw, Xn, Xs, Rs);
                    rQs[o1][0][tid] = X[0] + Rs[0];
                    rQs[o1][1][tid] = X[1] + Rs[1];
                    rQs[o1][2][tid] = X[2] + Rs[2];
                    if (POL) {
                        PT Pe[2] = {rP[a3][0][te], rP[a3][1][te]};
                        PT Pw[2] = {rP[a3][0][tw], rP[a3][1][tw]};
                        const int an = dhi ? a3 : a2;
                        PT Pn[2] = {rP[an][0][tid], rP[an][1][tid]};
                        PT Ps[2] = {dlo ? Pc[0] : cin.p0, dlo ? Pc[1] : cin.p1};
                        PT Rp[2];
                        rhs_P(S, cout.g, cout.hx, cout.hy, Pc, Pe, Pw, Pn, Ps, Rp);
                        rQp[o1][0][tid] = Pc[0] + Rp[0];
                        rQp[o1][1][tid] = Pc[1] + Rp[1];
                    }
                }
                cout.s0 = X[0];
                cout.s1 = X[1];
                cout.s2 = X[2];
                cout.p0 = Pc[0];
                cout.p1 = Pc[1];
            }

            // ---- stage E: corrector at row f-4 with the inputs stage D froze one iteration ago;
            // from j = 7 it records the predicted centre values as next iteration's south row
            if (j >= 7 && colE) {
                float X[3], Xe[3], Xw[3], Xn[3], Rs[3];
                PT Y[2], Ye[2], Yw[2], Yn[2], Rp[2];
#pragma unroll
                for (int q = 0; q < 3; ++q) X[q] = rQs[o0][q][tid];
                Y[0] = POL ? rQp[o0][0][tid] : (PT)0;
                Y[1] = POL ? rQp[o0][1][tid] : (PT)0;
                if (j >= 8) {
                    const bool elo = walls && rm4 == 0u, ehi = walls && rm4 == ytop;
                    const int on = ehi ? o0 : o1;
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        Xe[q] = rQs[o0][q][te];
                        Xw[q] = rQs[o0][q][tw];
                        Xn[q] = rQs[on][q][tid];
                    }
                    const float Xs[3] = {elo ? X[0] : cin.q0, elo ? X[1] : cin.q1, elo ? X[2] : cin.q2};
                    rhs_sigma(S, cin.k, cin.g, cin.hx, cin.hy, X, Xe, Xw, Xn, Xs, Rs);
                    const unsigned o = rm4 * nx * 4u, N4 = N * 4u;
                    buf_stf(rSo, b4, o, 0.5f * ((cin.s0 + X[0]) + Rs[0]));
                    buf_stf(rSo, b4, N4 + o, 0.5f * ((cin.s1 + X[1]) + Rs[1]));
                    buf_stf(rSo, b4, 2u * N4 + o, 0.5f * ((cin.s2 + X[2]) + Rs[2]));
                    if (POL) {   // without P both P buffers stay zero
#pragma unroll
                        for (int q = 0; q < 2; ++q) {
                            Ye[q] = rQp[o0][q][te];
                            Yw[q] = rQp[o0][q][tw];
                            Yn[q] = rQp[on][q][tid];
                        }
                        const PT Ys[2] = {elo ? Y[0] : cin.qp0, elo ? Y[1] : cin.qp1};
                        rhs_P(S, cin.g, cin.hx, cin.hy, Y, Ye, Yw, Yn, Ys, Rp);
                        const unsigned oP = rm4 * nx * (unsigned)sizeof(PT), NP = N * (unsigned)sizeof(PT);
                        buf_st(rPo, bP, oP, (PT)0.5 * ((cin.p0 + Y[0]) + Rp[0]));
                        buf_st(rPo, bP, NP + oP, (PT)0.5 * ((cin.p1 + Y[1]) + Rp[1]));
                    }
                }
                cout.q0 = X[0];
                cout.q1 = X[1];
                cout.q2 = X[2];
                cout.qp0 = Y[0];
                cout.qp1 = Y[1];
            }
            inc_row(rp1, ny);
            inc_row(r0, ny);
            inc_row(rm1, ny);
            inc_row(rm2, ny);
            inc_row(rm3, ny);
            inc_row(rm4, ny);
        };

        // two iterations per trip with the register sets swapped, so no values are copied.  The
        // waves' issue priority falls in thirds as the item progresses: a compute unit's SIMDs are
        // shared by several work-groups, and under the hardware's oldest-first arbitration the
        // last-dispatched ones would otherwise trail alone, at low VALU use, at the end.  When the
        // whole grid is one round of at most four work-groups per unit, dealt to the units in turn,
        // work-group b is the (b / cus)-th on its unit, and the later ones hold each priority three
        // row iterations longer per older work-group (longer grids start their work-groups as
        // others finish, and gain nothing from it).  Items that touch a body (their spread-force
        // reads make them the slowest) keep the top priority, so they no longer finish last.
        const int lag = (int)gridDim.x <= 4 * cus ? 3 * min(3, (int)blockIdx.x / cus) : 0;
        const int q1 = niter / 3 + lag, q2 = (2 * niter) / 3 + lag;
        for (int j = 2; j < niter; j += 2) {
            if (nib != 0)
                __builtin_amdgcn_s_setprio(3);
            else if (j >= q2)
                __builtin_amdgcn_s_setprio(0);
            else if (j >= q1)
                __builtin_amdgcn_s_setprio(1);
            else
                __builtin_amdgcn_s_setprio(2);
            iterate(j, preA, preB, carA, carB);
            if (j + 1 < niter) iterate(j + 1, preB, preA, carB, carA);
        }
    }
}

// ------------------------------------------------------------------------------------------------
// multi-pass reference step: one thread per site, intermediate fields in scratch planes
// ------------------------------------------------------------------------------------------------

// site indices of (x, y) and its four neighbours; with walls the row beyond a wall is the mirror
// ghost (the site itself: zero normal derivative), flagged in lo / hi for odd (no-slip) fields
struct Nb {
    size_t c, e, w, n, s;
    bool lo, hi, le, ri;   // the south, north, west, east neighbour is a wall ghost
};
// walls: 1 below row 0 and above row ny-1; 2 also left of column 0 and right of column nx-1
__device__ __forceinline__ Nb nbrs(int x, int y, int nx, int ny, int walls = 0) {
    Nb q;
    size_t row = (size_t)y * nx;
    q.c = row + x;
    q.le = walls == 2 && x == 0;
    q.ri = walls == 2 && x == nx - 1;
    q.e = q.ri ? q.c : row + wrapi(x + 1, nx);
    q.w = q.le ? q.c : row + wrapi(x - 1, nx);
    q.lo = walls && y == 0;
    q.hi = walls && y == ny - 1;
    q.n = q.hi ? q.c : (size_t)wrapi(y + 1, ny) * nx + x;
    q.s = q.lo ? q.c : (size_t)wrapi(y - 1, ny) * nx + x;
    return q;
}

__device__ __forceinline__ bool site_of(const SiteBlock *blk, const SimDev *sims, int &sim, int &x, int &y) {
    SiteBlock b = blk[blockIdx.x];
    const SimDev &S = sims[b.sim];
    int i = b.start + threadIdx.x;
    sim = b.sim;
    if (i >= S.nx * S.ny) return false;
    y = i / S.nx;
    x = i - y * S.nx;
    return true;
}

template <typename PT>
__global__ __launch_bounds__(256) void k_mp_sigE(const SimDev *__restrict__ sims, const SiteBlock *__restrict__ blk,
                                                 int cur, int *__restrict__ d_t) {
    if (d_t && blockIdx.x == 0 && threadIdx.x == 0) d_t[0] = d_t[0] + 1;
    int sim, x, y;
    if (!site_of(blk, sims, sim, x, y)) return;
    const SimDev &S = sims[sim];
    const size_t N = (size_t)S.nx * S.ny;
    const PT *P = static_cast<const PT *>(S.P[cur]);
    Nb q = nbrs(x, y, S.nx, S.ny, S.walls);
    PT Pc[2] = {P[q.c], P[N + q.c]}, Pe[2] = {P[q.e], P[N + q.e]}, Pw[2] = {P[q.w], P[N + q.w]};
    PT Pn[2] = {P[q.n], P[N + q.n]}, Ps[2] = {P[q.s], P[N + q.s]};
    float E[4];
    ericksen(S, Pc, Pe, Pw, Pn, Ps, E);
    for (int k = 0; k < 4; ++k) S.sE[k * N + q.c] = E[k];
}

// force at a site from the stress, the Ericksen scratch planes and the bodies
__device__ __forceinline__ void site_force(const SimDev &S, const BodyDev *bodies, int cur, int x, int y, const Nb &q,
                                           float &Fx, float &Fy, float &fpx, float &fpy) {
    const size_t N = (size_t)S.nx * S.ny;
    const float *sg = S.sig[cur];
    fpx = 0.5f * (sg[q.e] - sg[q.w]) + 0.5f * (sg[2 * N + q.n] - sg[2 * N + q.s]);
    fpy = 0.5f * (sg[2 * N + q.e] - sg[2 * N + q.w]) + 0.5f * (sg[N + q.n] - sg[N + q.s]);
    Fx = fpx + S.gx;
    Fy = fpy + S.gy;
    if (S.ericksen) {
        const float *E = S.sE;
        Fx += 0.5f * (E[q.e] - E[q.w]) + 0.5f * (E[N + q.n] - E[N + q.s]);
        Fy += 0.5f * (E[2 * N + q.e] - E[2 * N + q.w]) + 0.5f * (E[3 * N + q.n] - E[3 * N + q.s]);
    }
    if (S.nb) ib_force(S, bodies, cur, x, y, Fx, Fy);
}

template <typename HT>
__device__ __forceinline__ void pull_pops(const SimDev &S, const HT *hin, int x, int y, float d[9]) {
    const size_t N = (size_t)S.nx * S.ny;
#pragma unroll
    for (int n = 0; n < 9; ++n) {
        const int ys = y - kCY[n], xs = x - kCX[n];
        if ((S.walls && (ys < 0 || ys >= S.ny)) || (S.walls == 2 && (xs < 0 || xs >= S.nx))) {
            // halfway bounce-back: the opposite direction
            d[n] = Pop<HT>::load(hin, kOpp[n] * N + (size_t)y * S.nx + x, S.inv_scale);   // at this site
            continue;
        }
        size_t i = (size_t)wrapi(ys, S.ny) * S.nx + wrapi(xs, S.nx);
        d[n] = Pop<HT>::load(hin, n * N + i, S.inv_scale);
    }
}

template <typename HT>
__global__ __launch_bounds__(256) void k_mp_lb(const SimDev *__restrict__ sims, const BodyDev *__restrict__ bodies,
                                               const SiteBlock *__restrict__ blk, int cur) {
    int sim, x, y;
    if (!site_of(blk, sims, sim, x, y)) return;
    const SimDev &S = sims[sim];
    const size_t N = (size_t)S.nx * S.ny;
    Nb q = nbrs(x, y, S.nx, S.ny, S.walls);
    float Fx, Fy, fpx, fpy;
    site_force(S, bodies, cur, x, y, q, Fx, Fy, fpx, fpy);
    float d[9];
    pull_pops<HT>(S, reinterpret_cast<const HT *>(S.h[cur]), x, y, d);
    float drho, ux, uy;
    collide(d, Fx, Fy, S.omega, S.guo, drho, ux, uy);
    HT *hout = reinterpret_cast<HT *>(S.h[cur ^ 1]);
    for (int n = 0; n < 9; ++n) Pop<HT>::store(hout, n * N + q.c, d[n], S.scale);
    S.v[q.c] = ux;
    S.v[N + q.c] = uy;
    if (S.nb) ib_store_v(S, bodies, cur, x, y, ux, uy);
}

__device__ __forceinline__ Grad grad_at(const SimDev &S, const Nb &q) {
    const size_t N = (size_t)S.nx * S.ny;
    const float *v = S.v;
    // no-slip ghosts beyond a wall: the negated velocity of the wall row
    // (and half of it: grad_v takes v / 2)
    const float sn = q.hi ? -0.5f : 0.5f, ss = q.lo ? -0.5f : 0.5f, se = q.ri ? -0.5f : 0.5f, sw = q.le ? -0.5f : 0.5f;
    return grad_v(se * v[q.e], sw * v[q.w], sn * v[q.n], ss * v[q.s], se * v[N + q.e], sw * v[N + q.w], sn * v[N + q.n],
                  ss * v[N + q.s]);
}

__device__ __forceinline__ void gather3(const float *f, size_t N, const Nb &q, float X[3], float Xe[3], float Xw[3],
                                        float Xn[3], float Xs[3]) {
    for (int k = 0; k < 3; ++k) {
        X[k] = f[k * N + q.c];
        Xe[k] = f[k * N + q.e];
        Xw[k] = f[k * N + q.w];
        Xn[k] = f[k * N + q.n];
        Xs[k] = f[k * N + q.s];
    }
}
template <typename PT>
__device__ __forceinline__ void gather2(const PT *f, size_t N, const Nb &q, PT X[2], PT Xe[2], PT Xw[2], PT Xn[2],
                                        PT Xs[2]) {
    for (int k = 0; k < 2; ++k) {
        X[k] = f[k * N + q.c];
        Xe[k] = f[k * N + q.e];
        Xw[k] = f[k * N + q.w];
        Xn[k] = f[k * N + q.n];
        Xs[k] = f[k * N + q.s];
    }
}

template <typename PT>
__global__ __launch_bounds__(256) void k_mp_pred(const SimDev *__restrict__ sims, const SiteBlock *__restrict__ blk,
                                                 int cur) {
    int sim, x, y;
    if (!site_of(blk, sims, sim, x, y)) return;
    const SimDev &S = sims[sim];
    const size_t N = (size_t)S.nx * S.ny;
    Nb q = nbrs(x, y, S.nx, S.ny, S.walls);
    Grad g = grad_at(S, q);
    float hx = 0.5f * S.v[q.c], hy = 0.5f * S.v[N + q.c];
    float X[3], Xe[3], Xw[3], Xn[3], Xs[3], Rs[3];
    gather3(S.sig[cur], N, q, X, Xe, Xw, Xn, Xs);
    PT Y[2], Ye[2], Yw[2], Yn[2], Ys[2], Rp[2];
    gather2(static_cast<const PT *>(S.P[cur]), N, q, Y, Ye, Yw, Yn, Ys);
    Stiff k = stiffness(S, reinterpret_cast<const float4 *>(S.tab), (float)((PT)S.pref[0] + Y[0]),
                        (float)((PT)S.pref[1] + Y[1]));
    rhs_sigma(S, k, g, hx, hy, X, Xe, Xw, Xn, Xs, Rs);
    rhs_P(S, g, hx, hy, Y, Ye, Yw, Yn, Ys, Rp);
    for (int c = 0; c < 3; ++c) S.sps[c * N + q.c] = X[c] + Rs[c];
    PT *spp = static_cast<PT *>(S.spp);
    for (int c = 0; c < 2; ++c) spp[c * N + q.c] = Y[c] + Rp[c];
}

template <typename PT>
__global__ __launch_bounds__(256) void k_mp_corr(const SimDev *__restrict__ sims, const SiteBlock *__restrict__ blk,
                                                 int cur) {
    int sim, x, y;
    if (!site_of(blk, sims, sim, x, y)) return;
    const SimDev &S = sims[sim];
    const size_t N = (size_t)S.nx * S.ny;
    Nb q = nbrs(x, y, S.nx, S.ny, S.walls);
    Grad g = grad_at(S, q);
    float hx = 0.5f * S.v[q.c], hy = 0.5f * S.v[N + q.c];
    const PT *P = static_cast<const PT *>(S.P[cur]);
    Stiff k = stiffness(S, reinterpret_cast<const float4 *>(S.tab), (float)((PT)S.pref[0] + P[q.c]),
                        (float)((PT)S.pref[1] + P[N + q.c]));
    float X[3], Xe[3], Xw[3], Xn[3], Xs[3], Rs[3];
    gather3(S.sps, N, q, X, Xe, Xw, Xn, Xs);
    PT Y[2], Ye[2], Yw[2], Yn[2], Ys[2], Rp[2];
    gather2(static_cast<const PT *>(S.spp), N, q, Y, Ye, Yw, Yn, Ys);
    rhs_sigma(S, k, g, hx, hy, X, Xe, Xw, Xn, Xs, Rs);
    rhs_P(S, g, hx, hy, Y, Ye, Yw, Yn, Ys, Rp);
    const float *sg = S.sig[cur];
    float *so = S.sig[cur ^ 1];
    PT *Po = static_cast<PT *>(S.P[cur ^ 1]);
    for (int c = 0; c < 3; ++c) so[c * N + q.c] = 0.5f * ((sg[c * N + q.c] + X[c]) + Rs[c]);
    for (int c = 0; c < 2; ++c) Po[c * N + q.c] = (PT)0.5 * ((P[c * N + q.c] + Y[c]) + Rp[c]);
}

// ------------------------------------------------------------------------------------------------
// observables and reductions
// ------------------------------------------------------------------------------------------------

// planes of `out` (floats): drho, vx, vy, sxx, syy, sxy, Px, Py, fpx, fpy at the current time
template <typename HT>
__global__ __launch_bounds__(256) void k_readout(const SimDev *__restrict__ sims, const BodyDev *__restrict__ bodies,
                                                 const SiteBlock *__restrict__ blk, int cur, float *__restrict__ out) {
    int sim, x, y;
    if (!site_of(blk, sims, sim, x, y)) return;
    const SimDev &S = sims[sim];
    const size_t N = (size_t)S.nx * S.ny;
    Nb q = nbrs(x, y, S.nx, S.ny, S.walls);
    float Fx, Fy, fpx, fpy;
    site_force(S, bodies, cur, x, y, q, Fx, Fy, fpx, fpy);
    float d[9];
    pull_pops<HT>(S, reinterpret_cast<const HT *>(S.h[cur]), x, y, d);
    float drho, ux, uy;
    collide(d, Fx, Fy, S.omega, S.guo, drho, ux, uy);
    typedef typename PolOf<HT>::T PT;
    const float *sg = S.sig[cur];
    const PT *P = static_cast<const PT *>(S.P[cur]);
    out[0 * N + q.c] = drho;
    out[1 * N + q.c] = ux;
    out[2 * N + q.c] = uy;
    out[3 * N + q.c] = sg[q.c];
    out[4 * N + q.c] = sg[N + q.c];
    out[5 * N + q.c] = sg[2 * N + q.c];
    out[6 * N + q.c] = (float)((PT)S.pref[0] + P[q.c]);
    out[7 * N + q.c] = (float)((PT)S.pref[1] + P[N + q.c]);
    out[8 * N + q.c] = fpx;
    out[9 * N + q.c] = fpy;
}

// block partial sums (FP64) of drho and sum_n c_n d_n over the stored populations of one sim;
// the stored (post-collision, not yet streamed) populations have the same domain totals
template <typename HT>
__global__ __launch_bounds__(256) void k_sums(const SimDev *__restrict__ sims, int sim, int cur,
                                              double *__restrict__ partial) {
    __shared__ double sh[3][4];
    const SimDev &S = sims[sim];
    const size_t N = (size_t)S.nx * S.ny;
    const HT *h = reinterpret_cast<const HT *>(S.h[cur]);
    double m = 0.0, jx = 0.0, jy = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (size_t)gridDim.x * 256) {
        float d[9];
#pragma unroll
        for (int n = 0; n < 9; ++n) d[n] = Pop<HT>::load(h, n * N + i, S.inv_scale);
#pragma unroll
        for (int n = 0; n < 9; ++n) {
            m += (double)d[n];
            jx += (double)(kCX[n] * d[n]);
            jy += (double)(kCY[n] * d[n]);
        }
    }
    m = wave_sum(m);
    jx = wave_sum(jx);
    jy = wave_sum(jy);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        sh[0][wv] = m;
        sh[1][wv] = jx;
        sh[2][wv] = jy;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = (sh[threadIdx.x][0] + sh[threadIdx.x][1]) + (sh[threadIdx.x][2] + sh[threadIdx.x][3]);
        partial[3 * blockIdx.x + threadIdx.x] = s;
    }
}

// sum the block partials in a fixed order; out = (sum rho, momentum x, momentum y).  With
// check_mass > 0, raise the watchdog when the mass is not finite or drifts by more than 1e-6.
__global__ __launch_bounds__(64) void k_sums_final(const SimDev *__restrict__ sims, int sim, const double *__restrict__ partial,
                                                   int nblocks, double *__restrict__ out, double check_mass,
                                                   int *__restrict__ d_status) {
    const int lane = threadIdx.x;
    double a[3] = {0.0, 0.0, 0.0};
    for (int b = lane; b < nblocks; b += 64)
        for (int k = 0; k < 3; ++k) a[k] += partial[3 * b + k];
    for (int k = 0; k < 3; ++k) a[k] = wave_sum(a[k]);
    if (lane == 0) {
        const SimDev &S = sims[sim];
        double mass = (double)S.nx * (double)S.ny + a[0];
        out[0] = mass;
        out[1] = a[1];
        out[2] = a[2];
        if (check_mass > 0.0) {
            bool ok = isfinite(mass) && isfinite(a[1]) && isfinite(a[2]) && fabs(mass - check_mass) <= 1e-6 * check_mass;
            if (!ok) atomicOr(d_status, kStatusUnstable);
        }
    }
}

// Integral along the directed edge (xa, ya) -> (xb, yb), restricted to y0 <= y <= y1, of
// g(x) dy with g(x) = clamp(x, x0, x1) - x0.  Summed over a closed polygon this is, by Green's
// theorem, the signed area of the polygon inside the box [x0, x1] x [y0, y1].  g is piecewise
// linear along the edge, so the midpoint rule on the pieces between its kinks is exact.
__device__ __forceinline__ double edge_box(double xa, double ya, double xb, double yb, double x0, double x1,
                                           double y0, double y1) {
    const double lo = fmax(fmin(ya, yb), y0), hi = fmin(fmax(ya, yb), y1);
    if (!(hi > lo)) return 0.0;   // outside the band, or a horizontal edge
    const double s = (xb - xa) / (yb - ya);
    const double xl = xa + s * (lo - ya), xh = xa + s * (hi - ya);
    double ta = 0.0, tb = 0.0;
    if (xh != xl) {
        const double inv = 1.0 / (xh - xl);
        ta = fmin(fmax((x0 - xl) * inv, 0.0), 1.0);
        tb = fmin(fmax((x1 - xl) * inv, 0.0), 1.0);
        if (ta > tb) {
            const double u = ta;
            ta = tb;
            tb = u;
        }
    }
    auto g = [&](double t) { return fmin(fmax(xl + t * (xh - xl), x0), x1) - x0; };
    const double integral = ta * g(0.5 * ta) + (tb - ta) * g(0.5 * (ta + tb)) + (1.0 - tb) * g(0.5 * (tb + 1.0));
    return (yb > ya ? 1.0 : -1.0) * (hi - lo) * integral;
}

// body observables, one 256-thread block per body: restoring force as the sum of div sigma over
// the sites inside the node polygon (even-odd rule), centre of mass, total node force, and the
// area-weighted restoring force: the sum over sites of (area of the site's unit cell inside the
// polygon) * div sigma, which varies continuously with the node positions
__global__ __launch_bounds__(256) void k_body_force(const SimDev *__restrict__ sims, const BodyDev *__restrict__ bodies,
                                                    int body0, int cur, double *__restrict__ out_all) {
    __shared__ double2 sR[kMaxNodes];
    __shared__ double sh[9][4];
    const BodyDev &B = bodies[body0 + blockIdx.x];
    double *out = out_all + kBodyOut * blockIdx.x;
    const SimDev &S = sims[B.sim];
    const int n = B.n, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double2 *R = reinterpret_cast<const double2 *>(B.R[cur]);
    const double2 *Fn = reinterpret_cast<const double2 *>(B.fnode);
    double mnx = 1e300, mny = 1e300, mxx = -1e300, mxy = -1e300, cx = 0, cy = 0, fx = 0, fy = 0, ar = 0;
    for (int a = tid; a < n; a += 256) {
        double2 r = R[a], q = R[a == 0 ? n - 1 : a - 1];
        sR[a] = r;
        mnx = fmin(mnx, r.x);
        mny = fmin(mny, r.y);
        mxx = fmax(mxx, r.x);
        mxy = fmax(mxy, r.y);
        cx += r.x;
        cy += r.y;
        fx += Fn[a].x;
        fy += Fn[a].y;
        ar += q.x * r.y - r.x * q.y;
    }
    double v9[9] = {wave_min(mnx), wave_min(mny), wave_max(mxx), wave_max(mxy),
                    wave_sum(cx),  wave_sum(cy),  wave_sum(fx),  wave_sum(fy), wave_sum(ar)};
    if (lane == 0)
        for (int k = 0; k < 9; ++k) sh[k][wv] = v9[k];
    __syncthreads();
    mnx = fmin(fmin(sh[0][0], sh[0][1]), fmin(sh[0][2], sh[0][3]));
    mny = fmin(fmin(sh[1][0], sh[1][1]), fmin(sh[1][2], sh[1][3]));
    mxx = fmax(fmax(sh[2][0], sh[2][1]), fmax(sh[2][2], sh[2][3]));
    mxy = fmax(fmax(sh[3][0], sh[3][1]), fmax(sh[3][2], sh[3][3]));
    double scx = (sh[4][0] + sh[4][1]) + (sh[4][2] + sh[4][3]);
    double scy = (sh[5][0] + sh[5][1]) + (sh[5][2] + sh[5][3]);
    double sfx = (sh[6][0] + sh[6][1]) + (sh[6][2] + sh[6][3]);
    double sfy = (sh[7][0] + sh[7][1]) + (sh[7][2] + sh[7][3]);
    const double orient = (sh[8][0] + sh[8][1]) + (sh[8][2] + sh[8][3]) < 0.0 ? -1.0 : 1.0;
    __syncthreads();
    const size_t N = (size_t)S.nx * S.ny;
    const float *sg = S.sig[cur];
    auto divx = [&](const Nb &q) {
        return 0.5 * ((double)sg[q.e] - (double)sg[q.w]) + 0.5 * ((double)sg[2 * N + q.n] - (double)sg[2 * N + q.s]);
    };
    auto divy = [&](const Nb &q) {
        return 0.5 * ((double)sg[2 * N + q.e] - (double)sg[2 * N + q.w]) + 0.5 * ((double)sg[N + q.n] - (double)sg[N + q.s]);
    };
    // sites strictly inside (even-odd)
    double ax = 0.0, ay = 0.0;
    {
        const int x0 = (int)ceil(mnx), x1 = (int)floor(mxx), y0 = (int)ceil(mny), y1 = (int)floor(mxy);
        const int wdt = x1 - x0 + 1, hgt = y1 - y0 + 1;
        for (int i = tid; i < wdt * hgt; i += 256) {
            const int X = x0 + i % wdt, Y = y0 + i / wdt;
            bool in = false;
            for (int a = 0, b = n - 1; a < n; b = a++) {
                double xa = sR[a].x, ya = sR[a].y, xb = sR[b].x, yb = sR[b].y;
                if ((ya > Y) != (yb > Y) && X < (xb - xa) * (Y - ya) / (yb - ya) + xa) in = !in;
            }
            if (!in) continue;
            Nb q = nbrs(wrapi(X, S.nx), wrapi(Y, S.ny), S.nx, S.ny, S.walls);
            ax += divx(q);
            ay += divy(q);
        }
    }
    // every cell [X - 1/2, X + 1/2] x [Y - 1/2, Y + 1/2] the bounding box touches, weighted by area
    double bx = 0.0, by = 0.0;
    {
        const int x0 = (int)floor(mnx + 0.5), x1 = (int)ceil(mxx - 0.5), y0 = (int)floor(mny + 0.5),
                  y1 = (int)ceil(mxy - 0.5);
        const int wdt = x1 - x0 + 1, hgt = y1 - y0 + 1;
        for (int i = tid; i < wdt * hgt; i += 256) {
            const int X = x0 + i % wdt, Y = y0 + i / wdt;
            double w = 0.0;
            for (int a = 0, b = n - 1; a < n; b = a++)
                w += edge_box(sR[b].x, sR[b].y, sR[a].x, sR[a].y, X - 0.5, X + 0.5, Y - 0.5, Y + 0.5);
            w *= orient;
            if (w == 0.0) continue;
            Nb q = nbrs(wrapi(X, S.nx), wrapi(Y, S.ny), S.nx, S.ny, S.walls);
            bx += w * divx(q);
            by += w * divy(q);
        }
    }
    double red[4] = {wave_sum(ax), wave_sum(ay), wave_sum(bx), wave_sum(by)};
    if (lane == 0)
        for (int k = 0; k < 4; ++k) sh[k][wv] = red[k];
    __syncthreads();
    if (tid == 0) {
        out[0] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
        out[1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
        out[2] = scx / n;
        out[3] = scy / n;
        out[4] = sfx;
        out[5] = sfy;
        out[6] = (sh[2][0] + sh[2][1]) + (sh[2][2] + sh[2][3]);
        out[7] = (sh[3][0] + sh[3][1]) + (sh[3][2] + sh[3][3]);
    }
}

// convert host-prepared FP32 population offsets (already un-streamed) to the storage type
template <typename HT>
__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ src, HT *__restrict__ dst, size_t n, float scale) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) Pop<HT>::store(dst, i, src[i], scale);
}

// streaming copy of n16 16-byte words, the bandwidth ceiling the field kernel is measured against:
// each thread moves four words per trip, all four loads issued before the stores, and the grid
// strides over the buffer so every compute unit keeps several loads in flight
__global__ __launch_bounds__(256) void k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                     size_t n16) {
    const size_t stride = (size_t)gridDim.x * 1024;
    for (size_t base = (size_t)blockIdx.x * 1024 + threadIdx.x; base < n16; base += stride) {
        uint4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (base + 256 * k < n16) v[k] = src[base + 256 * k];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (base + 256 * k < n16) dst[base + 256 * k] = v[k];
    }
}

// ------------------------------------------------------------------------------------------------
// launch wrappers (host)
// ------------------------------------------------------------------------------------------------

hipError_t launch_ib(bool advance, int nbodies, int ntiles, hipStream_t st, const SimDev *sims, BodyDev *bodies,
                     const int2 *blk, int cur, const int *d_t, int *d_status) {
    if (nbodies <= 0) return hipSuccess;
    if (ntiles <= kIbOneLaunchTiles) {
        // few tiles: one launch, each block repeats its body's node update
        if (advance)
            k_ib_step<true><<<ntiles, 256, 0, st>>>(sims, bodies, blk, cur, d_t, d_status);
        else
            k_ib_step<false><<<ntiles, 256, 0, st>>>(sims, bodies, blk, cur, d_t, d_status);
    } else {
        if (advance)
            k_ib_nodes<true><<<nbodies, 256, 0, st>>>(sims, bodies, cur, d_t, d_status);
        else
            k_ib_nodes<false><<<nbodies, 256, 0, st>>>(sims, bodies, cur, d_t, d_status);
        k_ib_spread<<<ntiles, 256, 0, st>>>(bodies, blk, advance ? (cur ^ 1) : cur, d_status);
    }
    return hipGetLastError();
}

// the kernel for (work-group size, storage type, walls, polarization)
typedef void (*FusedFn)(const SimDev *, const BodyDev *, const WorkItem *, int, int, int *, int);
template <int T, typename HT>
static FusedFn fused_fn_t(bool walls, bool pol) {
    if (walls) return pol ? k_fused<T, HT, true, true> : k_fused<T, HT, true, false>;
    return pol ? k_fused<T, HT, false, true> : k_fused<T, HT, false, false>;
}
static FusedFn fused_fn(int T, bool fp16, bool walls, bool pol) {
    if (T == 64) return fp16 ? fused_fn_t<64, __half>(walls, pol) : fused_fn_t<64, float>(walls, pol);
    if (T == 128) return fp16 ? fused_fn_t<128, __half>(walls, pol) : fused_fn_t<128, float>(walls, pol);
    if (T == 256) return fp16 ? fused_fn_t<256, __half>(walls, pol) : fused_fn_t<256, float>(walls, pol);
    return nullptr;
}

hipError_t launch_fused(int T, bool fp16, bool walls, bool pol, int grid, hipStream_t st, const SimDev *sims,
                        const BodyDev *bodies, const WorkItem *items, int n_items, int cur, int *d_t, int cus) {
    FusedFn f = fused_fn(T, fp16, walls, pol);
    if (!f || cus < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(grid), dim3(T), 0, st, sims, bodies, items, n_items, cur, d_t, cus);
    return hipGetLastError();
}

int fused_blocks_per_cu(int T, bool fp16, bool walls, bool pol) {
    FusedFn f = fused_fn(T, fp16, walls, pol);
    int n = 0;
    hipError_t e = f ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, T, 0) : hipErrorInvalidValue;
    return e == hipSuccess && n > 0 ? n : 1;
}

hipError_t launch_multipass(bool fp16, int nblocks, hipStream_t st, const SimDev *sims, const BodyDev *bodies,
                            const SiteBlock *blk, int cur, int *d_t) {
    if (fp16) {
        k_mp_sigE<float><<<nblocks, 256, 0, st>>>(sims, blk, cur, d_t);
        k_mp_lb<__half><<<nblocks, 256, 0, st>>>(sims, bodies, blk, cur);
        k_mp_pred<float><<<nblocks, 256, 0, st>>>(sims, blk, cur);
        k_mp_corr<float><<<nblocks, 256, 0, st>>>(sims, blk, cur);
    } else {
        k_mp_sigE<double><<<nblocks, 256, 0, st>>>(sims, blk, cur, d_t);
        k_mp_lb<float><<<nblocks, 256, 0, st>>>(sims, bodies, blk, cur);
        k_mp_pred<double><<<nblocks, 256, 0, st>>>(sims, blk, cur);
        k_mp_corr<double><<<nblocks, 256, 0, st>>>(sims, blk, cur);
    }
    return hipGetLastError();
}

hipError_t launch_readout(bool fp16, int nblocks, int block0, hipStream_t st, const SimDev *sims, const BodyDev *bodies,
                          const SiteBlock *blk, int cur, float *out) {
    if (fp16)
        k_mp_sigE<float><<<nblocks, 256, 0, st>>>(sims, blk + block0, cur, nullptr);
    else
        k_mp_sigE<double><<<nblocks, 256, 0, st>>>(sims, blk + block0, cur, nullptr);
    if (fp16)
        k_readout<__half><<<nblocks, 256, 0, st>>>(sims, bodies, blk + block0, cur, out);
    else
        k_readout<float><<<nblocks, 256, 0, st>>>(sims, bodies, blk + block0, cur, out);
    return hipGetLastError();
}

hipError_t launch_sums(bool fp16, int sim, int nblocks, hipStream_t st, const SimDev *sims, int cur, double *partial,
                       double *out, double check_mass, int *d_status) {
    if (fp16)
        k_sums<__half><<<nblocks, 256, 0, st>>>(sims, sim, cur, partial);
    else
        k_sums<float><<<nblocks, 256, 0, st>>>(sims, sim, cur, partial);
    k_sums_final<<<1, 64, 0, st>>>(sims, sim, partial, nblocks, out, check_mass, d_status);
    return hipGetLastError();
}

hipError_t launch_body_force(hipStream_t st, const SimDev *sims, const BodyDev *bodies, int body0, int nbodies, int cur,
                             double *out) {
    if (nbodies <= 0) return hipSuccess;
    k_body_force<<<nbodies, 256, 0, st>>>(sims, bodies, body0, cur, out);
    return hipGetLastError();
}

hipError_t launch_stream_copy(hipStream_t st, const void *src, void *dst, size_t bytes) {
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n16 + 1023) / 1024, 256 * 16);
    k_stream_copy<<<(unsigned)blocks, 256, 0, st>>>(static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n16);
    return hipGetLastError();
}

hipError_t launch_pack(bool fp16, hipStream_t st, const float *src, void *dst, size_t n, float scale) {
    int nb = (int)((n + 255) / 256);
    if (fp16)
        k_pack<__half><<<nb, 256, 0, st>>>(src, reinterpret_cast<__half *>(dst), n, scale);
    else
        k_pack<float><<<nb, 256, 0, st>>>(src, reinterpret_cast<float *>(dst), n, scale);
    return hipGetLastError();
}

}  // namespace lbk
