// Device-side arithmetic of one lattice site, shared by the fused and multi-pass kernels.
//
// Populations are stored as offsets from the rest weights, d_n = h_n - w_n (FP32 arithmetic;
// FP32 or FP16-times-2^S storage).  Every right-hand side takes time-t inputs (Fig. 2 caption).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <type_traits>

#include "lb_common.h"

namespace lbk {

// global address space: loads and stores through these pointers compile to global_* instructions
// (flat ones would also count against the LDS wait counter and serialise the row prefetch)
#define LBK_GLOBAL __attribute__((address_space(1)))

template <typename T> __device__ __forceinline__ const LBK_GLOBAL T *gptr(const T *p) {
    return (const LBK_GLOBAL T *)p;
}
template <typename T> __device__ __forceinline__ LBK_GLOBAL T *gptr(T *p) { return (LBK_GLOBAL T *)p; }

// D2Q9: rest, +x, +y, -x, -y, (+,+), (-,+), (-,-), (+,-)
__device__ constexpr int kCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kCY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};   // c_kOpp[n] = -c_n
__device__ constexpr float kW[9] = {4.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f,
                                    1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};

__device__ __forceinline__ int wrapi(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// ---- population storage -----------------------------------------------------------------
template <typename HT> struct Pop;
// every state array of one simulation is < 4 GiB (lb_create limits a lattice to 1e8 sites), so
// an unsigned 32-bit element index from a uniform base addresses it
// byte offset of element i, kept in 32 bits so the address is scalar base + 32-bit vector offset
template <typename T> __device__ __forceinline__ const LBK_GLOBAL T *at32(const T *base, unsigned i) {
    return (const LBK_GLOBAL T *)((const LBK_GLOBAL char *)base + i * (unsigned)sizeof(T));
}
template <typename T> __device__ __forceinline__ LBK_GLOBAL T *at32(T *base, unsigned i) {
    return (LBK_GLOBAL T *)((LBK_GLOBAL char *)base + i * (unsigned)sizeof(T));
}

// Raw buffer access to a state array: a buffer resource over its base (no stride, the whole 32-bit
// range, the gfx9 raw-buffer format word), a lane's byte offset (its column) in the vector offset
// and the uniform part (plane and row) in the scalar offset, so a load or store costs no vector
// arithmetic.  Every state array of one simulation is < 4 GiB, so both offsets fit 32 bits.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t state_rsrc(const void *p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)0xffffffff, 0x00020000);
}
__device__ __forceinline__ float buf_ldf(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void buf_stf(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float &v) {
    v = buf_ldf(r, voff, soff);
}
__device__ __forceinline__ void buf_ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double &v) {
    v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v) {
    buf_stf(r, voff, soff, v);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double v) {
    typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)) B64;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B64, v), r, (int)voff, (int)soff, 0);
}

// Raw: the stored word, fetched one iteration ahead and converted only when used, so a prefetch
// does not wait for its own load.
template <> struct Pop<float> {
    typedef float Raw;
    static __device__ __forceinline__ Raw ld_raw(const float *p, unsigned i) { return *at32(p, i); }
    static __device__ __forceinline__ float cvt(Raw r, float) { return r; }
    static __device__ __forceinline__ float load(const float *p, size_t i, float) { return p[i]; }
    static __device__ __forceinline__ void store(float *p, size_t i, float v, float) { p[i] = v; }
    static __device__ __forceinline__ float ld(const float *p, unsigned i, float) { return *at32(p, i); }
    static __device__ __forceinline__ void st(float *p, unsigned i, float v, float) { *at32(p, i) = v; }
    // the stored value as is (for FP16 storage: still times the 2^S scale)
    static __device__ __forceinline__ float cvt_stored(Raw r) { return r; }
    static __device__ __forceinline__ void st_stored(float *p, unsigned i, float v) { *at32(p, i) = v; }
    static __device__ __forceinline__ Raw ld_buf(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
        return buf_ldf(r, voff, soff);
    }
    static __device__ __forceinline__ void st_buf(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v) {
        buf_stf(r, voff, soff, v);
    }
    static constexpr bool kScaled = false;
};
template <> struct Pop<__half> {
    // a 32-bit word per value: 16-bit values would be packed in pairs, which waits for both loads
    typedef unsigned Raw;
    static __device__ __forceinline__ Raw ld_raw(const __half *p, unsigned i) {
        return *at32(reinterpret_cast<const unsigned short *>(p), i);
    }
    static __device__ __forceinline__ float cvt(Raw r, float inv_scale) {
        return __half2float(__ushort_as_half((unsigned short)r)) * inv_scale;
    }
    static __device__ __forceinline__ float load(const __half *p, size_t i, float inv_scale) {
        return __half2float(p[i]) * inv_scale;
    }
    static __device__ __forceinline__ void store(__half *p, size_t i, float v, float scale) {
        p[i] = __float2half_rn(v * scale);
    }
    static __device__ __forceinline__ float ld(const __half *p, unsigned i, float inv_scale) {
        return __half2float(__ushort_as_half(*at32(reinterpret_cast<const unsigned short *>(p), i))) * inv_scale;
    }
    static __device__ __forceinline__ void st(__half *p, unsigned i, float v, float scale) {
        *at32(reinterpret_cast<unsigned short *>(p), i) = __half_as_ushort(__float2half_rn(v * scale));
    }
    static __device__ __forceinline__ float cvt_stored(Raw r) { return __half2float(__ushort_as_half((unsigned short)r)); }
    static __device__ __forceinline__ void st_stored(__half *p, unsigned i, float v) {
        *at32(reinterpret_cast<unsigned short *>(p), i) = __half_as_ushort(__float2half_rn(v));
    }
    static __device__ __forceinline__ Raw ld_buf(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
        return (unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
    }
    static __device__ __forceinline__ void st_buf(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(v)), r, (int)voff, (int)soff, 0);
    }
    static constexpr bool kScaled = true;
};

// ---- BGK collision with Guo forcing (eqBGK, Sec. II B force coupling) --------------------
// In: pre-collision offsets d[9], force F.  Out: post-collision offsets in d, and the
// force-corrected velocity u = (sum c h + F/2)/rho, drho = rho - 1.  SCALED: d in and out are
// the offsets times `scale`, the power of two of the FP16 storage, so the stored words are
// converted without a multiply (every rescaling by a power of two is exact).
template <bool SCALED>
__device__ __forceinline__ void collide_t(float d[9], float Fx, float Fy, float omega, float guo, float scale,
                                          float inv_scale, float &drho, float &ux, float &uy) {
    const float up = d[5] + d[6], dn = d[7] + d[8];   // the diagonal pairs with c_y = +1, -1
    drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + up) + dn);
    float jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
    float jy = (d[2] - d[4]) + (up - dn);
    if (SCALED) {   // offsets held times the power-of-two storage scale: exact rescaling
        drho *= inv_scale;
        jx = fmaf(jx, inv_scale, 0.5f * Fx);
        jy = fmaf(jy, inv_scale, 0.5f * Fy);
    } else {
        jx += 0.5f * Fx;
        jy += 0.5f * Fy;
    }
    float rho = 1.0f + drho;
    float ir = __builtin_amdgcn_rcpf(rho);   // 1 ulp; rho is within a few per cent of 1
    ux = jx * ir;
    uy = jy * ir;
    // d' = (1 - omega) d + omega deq + src with, per direction n (t = c_n.u, g = c_n.F),
    //   deq = w_n (drho + rho (3 t + 4.5 t^2 - 1.5 u.u)),  src = guo w_n (3 (g - u.F) + 9 t g),
    // gathered as w_n (C0 + t (a1 + a2 t) + g (b1 + b2 t)) with per-site a1, a2, C0.  Opposite
    // directions share t^2 and t g and flip t and g, so each pair takes the even part
    // E = C0 + t (a2 t + b2 g) and the odd part O = a1 t + b1 g once: w_n (E + O) and w_n (E - O).
    const float uu15 = 1.5f * (ux * ux + uy * uy);
    const float uF = ux * Fx + uy * Fy;
    const float orho = omega * rho;
    const float a1 = 3.0f * orho, a2 = 4.5f * orho, b1 = 3.0f * guo, b2 = 9.0f * guo;
    const float C0 = omega * drho - orho * uu15 - b1 * uF;
    const float keep = 1.0f - omega;
    const float ws = SCALED ? kW[1] * scale : kW[1], wd = SCALED ? kW[5] * scale : kW[5];
    d[0] = fmaf(keep, d[0], (SCALED ? kW[0] * scale : kW[0]) * C0);
    auto pair = [&](int n, int m, float t, float g, float w) {   // m: the direction opposite to n
        const float E = fmaf(t, fmaf(a2, t, b2 * g), C0);
        const float O = fmaf(a1, t, b1 * g);
        const float wE = w * E, wO = w * O;
        d[n] = fmaf(keep, d[n], wE + wO);
        d[m] = fmaf(keep, d[m], wE - wO);
    };
    pair(1, 3, ux, Fx, ws);
    pair(2, 4, uy, Fy, ws);
    pair(5, 7, ux + uy, Fx + Fy, wd);
    pair(6, 8, uy - ux, Fy - Fx, wd);
}

__device__ __forceinline__ void collide(float d[9], float Fx, float Fy, float omega, float guo,
                                        float &drho, float &ux, float &uy) {
    collide_t<false>(d, Fx, Fy, omega, guo, 1.0f, 1.0f, drho, ux, uy);
}

// ---- stiffness C~(P) (App. B) via piecewise cubics of a2/s and a4/s^2 in s = |P|^2 ---------
// a2 cos(2 th) = A2 (Px^2 - Py^2), a2 sin(2 th) = A2 2 Px Py, and the same for a4 with the
// squares of those harmonics, so no angle and no division by |P| are needed.  The operator on
// plain components (Xxx, Xyy, Xxy) is
//   C11 = (S1 + X1 + 4 X2) / 8, C22 = C11 - X2, C12 = (S2 - X1) / 8, C33 = (S3 - X1) / 4,
//   C13 = (Y1 + 2 Y2) / 4, C23 = (2 Y2 - Y1) / 4,   C31 = C13 / 2, C32 = C23 / 2,
// with X1 = a4 cos 4th cA, X2 = a2 cos 2th cB, Y1 = a4 sin 4th cA, Y2 = a2 sin 2th cB and the
// isotropic parts S1, S2, S3 (SimDev holds S1 / 8, S2 / 8, S3 / 4); Stiff holds the angular ones
// pre-scaled: p = X1 / 8, q = X2 / 2, r = Y1 / 4, w = Y2 / 2.
struct Stiff {
    float p, q, r, w;
};

// tab: kStiffSeg segments x two float4 (cubic coefficients c0..c3 of A2, then of A4), in LDS or
// global memory
template <typename Tab>
__device__ __forceinline__ Stiff stiffness(const SimDev &S, Tab tab, float Px, float Py) {
    float sx = Px * Px, sy = Py * Py;
    float s = sx + sy;
    float A2, A4;
    if (s < S.smax) {
        float u = s * S.inv_ds;
        int i = min((int)u, kStiffSeg - 1);
        float t = u - (float)i;
        const float4 a = tab[2 * i], b = tab[2 * i + 1];
        A2 = fmaf(fmaf(fmaf(a.w, t, a.z), t, a.y), t, a.x);
        A4 = fmaf(fmaf(fmaf(b.w, t, b.z), t, b.y), t, b.x);
    } else {
        float r = S.smax * __builtin_amdgcn_rcpf(s);   // s >= smax > 0
        A2 = S.A2max * r;
        A4 = S.A4max * r * r;
    }
    float dd = sx - sy, ee = 2.0f * Px * Py;
    Stiff k;
    k.p = A4 * (dd * dd - ee * ee) * S.cA8;
    k.r = A4 * (dd * ee) * S.cA2;
    k.q = A2 * dd * S.cB2;
    k.w = A2 * ee * S.cB2;
    return k;
}

// y = C~ x on plain components (xx, yy, xy)
__device__ __forceinline__ void stiff_apply(const SimDev &S, const Stiff &k, float a, float b, float c,
                                            float &o0, float &o1, float &o2) {
    float C11 = (S.s1 + k.p) + k.q;
    float C22 = fmaf(-2.0f, k.q, C11);
    float C12 = S.s2 - k.p;
    float C33 = fmaf(-2.0f, k.p, S.s3);
    float C13 = k.r + k.w;
    float C23 = k.w - k.r;
    o0 = C11 * a + C12 * b + C13 * c;
    o1 = C12 * a + C22 * b + C23 * c;
    o2 = 0.5f * (C13 * a + C23 * b) + C33 * c;
}

// velocity gradient pieces at a site from central differences of HALF the velocity (h = v / 2 at
// the four neighbours), so the differences need no halving
struct Grad {
    float psi0, psi1, psi2, om;   // Psi_xx, Psi_yy, Psi_xy, Omega_xy
};

__device__ __forceinline__ Grad grad_v(float hxe, float hxw, float hxn, float hxs,
                                       float hye, float hyw, float hyn, float hys) {
    const float gxy = hye - hyw, gyx = hxn - hxs;   // d_x v_y, d_y v_x
    Grad g;
    g.psi0 = hxe - hxw;
    g.psi1 = hyn - hys;
    g.psi2 = 0.5f * (gxy + gyx);
    g.om = 0.5f * (gxy - gyx);
    return g;
}

// right-hand side of eqStiffCons (corotational derivative) for one component set:
// -(v.grad)X - (Omega X - X Omega) + C~(Psi - X/eta_p) + D_p lap X.
// X[c] centre, e/w/n/s neighbours of each component.
// hx, hy: half the velocity.  The advection and diffusion terms are one five-point stencil,
// D lap X - (v.grad) X = (D - hx) Xe + (D + hx) Xw + (D - hy) Xn + (D + hy) Xs - 4 D X, whose
// weights are shared by the three components.
__device__ __forceinline__ void rhs_sigma(const SimDev &S, const Stiff &k, const Grad &g, float hx, float hy,
                                          const float X[3], const float Xe[3], const float Xw[3],
                                          const float Xn[3], const float Xs[3], float R[3]) {
    float a = g.psi0 - S.inv_eta * X[0];
    float b = g.psi1 - S.inv_eta * X[1];
    float c = g.psi2 - S.inv_eta * X[2];
    float C0, C1, C2;
    stiff_apply(S, k, a, b, c, C0, C1, C2);
    const float J0 = 2.0f * g.om * X[2];
    const float J2 = g.om * (X[1] - X[0]);
    const float Bv[3] = {C0 - J0, C1 + J0, C2 - J2};
    const float we = S.D - hx, ww = S.D + hx, wn = S.D - hy, ws = S.D + hy;
#pragma unroll
    for (int q = 0; q < 3; ++q)
        R[q] = fmaf(we, Xe[q], fmaf(ww, Xw[q], fmaf(wn, Xn[q], fmaf(ws, Xs[q], fmaf(S.m4D, X[q], Bv[q])))));
}

// Polarization storage follows the population storage.  With FP32 populations (the full-precision
// form, bar 1e-4) P is FP64 state: its per-step increments can fall far below the FP32
// resolution of |P| ~ 1, and FP32 state rounding (3e-8 per step) feeds the molecular field a
// site-to-site noise that, through the Ericksen stress, measurably moves weak flows.  With FP16
// populations (the reduced-precision form, bar 1e-3) P is stored as FP32 offsets Y = P - pref
// from a per-simulation reference (the mean of the initial field), which keeps near-uniform
// director fields' offsets small and their increments resolved.  PT is the storage type; the FP64
// form takes pref = 0.
template <typename HT> struct PolOf { typedef double T; };
template <> struct PolOf<__half> { typedef float T; };

// Local quantities of eqBE and the Ericksen stress from the stored values.  The slope
// a = alpha + beta |P|^2 cancels to near zero at the equilibrium magnitude, so it is formed in FP64
// from the exact value pref + Y (formed in FP32 from the rounded centre value it feeds a noise
// into the molecular field that moves a 1000-step FP16 run by several 1e-3); the neighbour
// differences are formed in the storage precision (exact for FP64, exact for FP32 offsets of
// close neighbours) and the rest in FP32.
struct PLocal {
    float c[2];      // centre P = pref + Y
    float d[4][2];   // e, w, n, s minus the centre
    float a;         // alpha + beta |P|^2
};
template <typename PT>
__device__ __forceinline__ PLocal p_local(const SimDev &S, const PT Y[2], const PT Ye[2], const PT Yw[2],
                                          const PT Yn[2], const PT Ys[2]) {
    PLocal L;
    const double P0 = S.pref_d[0] + (double)Y[0], P1 = S.pref_d[1] + (double)Y[1];
    L.a = (float)fma(S.beta_d, fma(P0, P0, P1 * P1), S.alpha_d);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        L.c[q] = (float)((PT)S.pref[q] + Y[q]);
        L.d[0][q] = (float)(Ye[q] - Y[q]);
        L.d[1][q] = (float)(Yw[q] - Y[q]);
        L.d[2][q] = (float)(Yn[q] - Y[q]);
        L.d[3][q] = (float)(Ys[q] - Y[q]);
    }
    return L;
}

// right-hand side of eqBE for the stored offsets: -(v.grad)Y - Omega P + xi Psi P - Gamma h(P),
// h = (alpha + beta |P|^2) P - kappa lap P (pref is constant, so the gradients of P are those of Y).
// The advection and the Gamma kappa lap P part of -Gamma h are one stencil on the neighbour
// differences: (Gk - hx) de + (Gk + hx) dw + (Gk - hy) dn + (Gk + hy) ds, Gk = Gamma kappa.
template <typename PT>
__device__ __forceinline__ void rhs_P(const SimDev &S, const Grad &g, float hx, float hy, const PT Y[2],
                                      const PT Ye[2], const PT Yw[2], const PT Yn[2], const PT Ys[2], PT R[2]) {
    const PLocal L = p_local(S, Y, Ye, Yw, Yn, Ys);
    const float we = S.gk - hx, ww = S.gk + hx, wn = S.gk - hy, ws = S.gk + hy;
    const float ga = S.Gamma * L.a;
    float T[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) T[q] = fmaf(we, L.d[0][q], fmaf(ww, L.d[1][q], fmaf(wn, L.d[2][q], ws * L.d[3][q])));
    R[0] = (PT)fmaf(S.xi, fmaf(g.psi0, L.c[0], g.psi2 * L.c[1]), fmaf(-g.om, L.c[1], fmaf(-ga, L.c[0], T[0])));
    R[1] = (PT)fmaf(S.xi, fmaf(g.psi2, L.c[0], g.psi1 * L.c[1]), fmaf(g.om, L.c[0], fmaf(-ga, L.c[1], T[1])));
}

// Ericksen stress at a site (Sec. II C 1, with kappa on the gradient term), from the stored
// values: out = (xx, xy, yx, yy)
template <typename PT>
__device__ __forceinline__ void ericksen(const SimDev &S, const PT P[2], const PT Pe[2], const PT Pw[2],
                                         const PT Pn[2], const PT Ps[2], float E[4]) {
    const PLocal L = p_local(S, P, Pe, Pw, Pn, Ps);
    const float kap = S.kappa, xi = S.xi, P0 = L.c[0], P1 = L.c[1];
    const float lap0 = (L.d[0][0] + L.d[1][0]) + (L.d[2][0] + L.d[3][0]);
    const float lap1 = (L.d[0][1] + L.d[1][1]) + (L.d[2][1] + L.d[3][1]);
    const float hx = L.a * P0 - kap * lap0;
    const float hy = L.a * P1 - kap * lap1;
    // twice the central differences; kappa / 4 takes the halves
    const float dxPx = L.d[0][0] - L.d[1][0], dyPx = L.d[2][0] - L.d[3][0];
    const float dxPy = L.d[0][1] - L.d[1][1], dyPy = L.d[2][1] - L.d[3][1];
    const float anti = -0.5f * (P0 * hy - hx * P1);
    const float sym = 0.5f * xi * (P0 * hy + hx * P1);
    const float gxy = S.kap4 * (dxPx * dyPx + dxPy * dyPy);
    E[0] = xi * P0 * hx - S.kap4 * (dxPx * dxPx + dxPy * dxPy);
    E[1] = anti + sym - gxy;
    E[2] = -anti + sym - gxy;
    E[3] = xi * P1 * hy - S.kap4 * (dyPx * dyPx + dyPy * dyPy);
}

// (x - o) mod n for |x - o| < 2n, without an integer division
__device__ __forceinline__ int wrap_near(int d, int n) {
    d = d < 0 ? d + n : d;
    return d >= n ? d - n : d;
}

// immersed-boundary force at lattice site (x, y) from the bodies' spread-force patches
__device__ __forceinline__ void ib_force(const SimDev &S, const BodyDev *bodies, int parity, int x, int y,
                                         float &Fx, float &Fy) {
    for (int b = 0; b < S.nb; ++b) {
        const BodyDev &B = bodies[S.b0 + b];
        int px = wrap_near(x - gptr(B.origin)[4 * parity + 2], S.nx);
        int py = wrap_near(y - gptr(B.origin)[4 * parity + 3], S.ny);
        if ((unsigned)px < (unsigned)B.ps && (unsigned)py < (unsigned)B.ps) {
            unsigned i = (unsigned)(py * B.ps + px);
            Fx += gptr(B.fib)[i];
            Fy += gptr(B.fib)[(unsigned)(B.ps * B.ps) + i];
        }
    }
}

// store the fluid velocity into the bodies' velocity patches (read by the node update)
__device__ __forceinline__ void ib_store_v(const SimDev &S, const BodyDev *bodies, int parity, int x, int y,
                                           float ux, float uy) {
    for (int b = 0; b < S.nb; ++b) {
        const BodyDev &B = bodies[S.b0 + b];
        int px = wrap_near(x - gptr(B.origin)[4 * parity + 2], S.nx);
        int py = wrap_near(y - gptr(B.origin)[4 * parity + 3], S.ny);
        if ((unsigned)px < (unsigned)B.ps && (unsigned)py < (unsigned)B.ps) {
            unsigned i = (unsigned)(py * B.ps + px);
            gptr(B.vib)[i] = ux;
            gptr(B.vib)[(unsigned)(B.ps * B.ps) + i] = uy;
        }
    }
}

// A body whose force/velocity patch touches a fused work item: the wrapped patch origin at the
// current parity, the patch side and the patch planes.
struct ItemBody {
    int ox, oy, ps, pad;
    const float *fib;
    float *vib;
};

// do the periodic intervals [a, a + la) and [b, b + lb) on a ring of n sites intersect?
// (0 <= a, b < n)
__device__ __forceinline__ bool ring_overlap(int a, int la, int b, int lb, int n) {
    if (la >= n || lb >= n) return true;
    int d = b - a;
    d = d < 0 ? d + n : d;
    if (d < la) return true;
    int e = a - b;
    e = e < 0 ? e + n : e;
    return e < lb;
}

__device__ __forceinline__ void ib_force_list(const ItemBody *L, int n, int nx, int ny, int x, int y, float &Fx,
                                              float &Fy) {
    for (int k = 0; k < n; ++k) {
        const ItemBody &B = L[k];
        int px = wrap_near(x - B.ox, nx), py = wrap_near(y - B.oy, ny);
        if ((unsigned)px < (unsigned)B.ps && (unsigned)py < (unsigned)B.ps) {
            unsigned i = (unsigned)(py * B.ps + px);
            Fx += gptr(B.fib)[i];
            Fy += gptr(B.fib)[(unsigned)(B.ps * B.ps) + i];
        }
    }
}

__device__ __forceinline__ void ib_store_v_list(const ItemBody *L, int n, int nx, int ny, int x, int y, float ux,
                                                float uy) {
    for (int k = 0; k < n; ++k) {
        const ItemBody &B = L[k];
        int px = wrap_near(x - B.ox, nx), py = wrap_near(y - B.oy, ny);
        if ((unsigned)px < (unsigned)B.ps && (unsigned)py < (unsigned)B.ps) {
            unsigned i = (unsigned)(py * B.ps + px);
            gptr(B.vib)[i] = ux;
            gptr(B.vib)[(unsigned)(B.ps * B.ps) + i] = uy;
        }
    }
}

// loads and stores at base + idx with a 32-bit byte offset (planes are < 4 GiB), so the address
// is a scalar base plus one vector register
template <typename T> __device__ __forceinline__ T ld32(const T *base, unsigned idx) { return *at32(base, idx); }
template <typename T> __device__ __forceinline__ void st32(T *base, unsigned idx, T v) { *at32(base, idx) = v; }

}  // namespace lbk
