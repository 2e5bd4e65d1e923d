// Host runtime and C-ABI of liblb (declared in include/lb.h).
//
// The caller owns one device arena; lb_create carves every buffer out of it (state ping-pong
// planes, stiffness tables, body patches, scratch), builds the work tables for the kernels and
// uploads the initial state.  lb_step queues kernels (optionally replaying a captured hipGraph);
// synchronising calls report deferred device errors and the watchdog.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lb.h"
#include "lb_common.h"
#include "lb_launch.h"

using namespace lbk;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(LB_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------------------------
// stiffness tables: a2/s and a4/s^2 of the von Mises closure on a uniform grid in s = |P|^2.
// The moments a_n(k) = <cos n theta> of g(theta; k) ~ exp(k cos theta) (Sec. II C 3) are
// evaluated by the trapezoid rule on a periodic grid (spectrally accurate), and k(P) solves
// <cos theta> = P by Newton's method with d<cos>/dk = <cos^2> - <cos>^2.
// ---------------------------------------------------------------------------------------------

struct VonMises {
    static constexpr int M = 1024;
    std::vector<double> c1, c2, c4;
    VonMises() : c1(M), c2(M), c4(M) {
        for (int j = 0; j < M; ++j) {
            double th = 2.0 * M_PI * j / M;
            c1[j] = std::cos(th);
            c2[j] = std::cos(2.0 * th);
            c4[j] = std::cos(4.0 * th);
        }
    }
    // moments <cos theta>, <cos 2 theta>, <cos 4 theta>
    void moments(double k, double &m1, double &m2, double &m4) const {
        double z = 0, a = 0, b = 0, c = 0;
        for (int j = 0; j < M; ++j) {
            double w = std::exp(k * (c1[j] - 1.0));
            z += w;
            a += w * c1[j];
            b += w * c2[j];
            c += w * c4[j];
        }
        m1 = a / z;
        m2 = b / z;
        m4 = c / z;
    }
    double k_of_p(double p) const {
        if (p <= 0.0) return 0.0;
        // start: approximate inverse k ~ p (2 - p^2)/(1 - p^2) (Banerjee et al. 2005)
        double k = p * (2.0 - p * p) / (1.0 - p * p), lo = 0.0, hi = 4.0 * k + 10.0;
        for (int it = 0; it < 100; ++it) {
            double m1, m2, m4;
            moments(k, m1, m2, m4);
            double f = m1 - p;
            if (f > 0) hi = k; else lo = k;
            double df = 0.5 * (1.0 + m2) - m1 * m1;
            double kn = k - f / df;
            if (!(kn > lo && kn < hi)) kn = 0.5 * (lo + hi);
            bool done = std::fabs(kn - k) <= 1e-14 * std::max(1.0, k);
            k = kn;
            if (done) break;
        }
        return k;
    }
};

struct Table {
    std::vector<float> coef;   // kStiffSeg segments x (A2: c0..c3, A4: c0..c3)
    double A2max, A4max;
};

// a2/s and a4/s^2 on kStiffSeg equal segments of s in [0, P_clamp^2], each a cubic in the local
// coordinate t in [0, 1] interpolating the exact values at the four Chebyshev points of the
// segment (within a factor of two of the best cubic; 64 segments give < 1e-7 relative error).
const Table &stiffness_table(double P_clamp) {
    static std::mutex mu;
    static std::map<double, Table> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(P_clamp);
    if (it != cache.end()) return it->second;
    static const VonMises vm;
    const double smax = P_clamp * P_clamp, ds = smax / kStiffSeg;
    auto values = [&](double s, double &A2, double &A4) {
        double k = vm.k_of_p(std::sqrt(s));
        double m1, m2, m4;
        vm.moments(k, m1, m2, m4);
        A2 = m2 / s;
        A4 = m4 / (s * s);
    };
    Table t;
    t.coef.resize(8 * kStiffSeg);
    for (int i = 0; i < kStiffSeg; ++i) {
        double tn[4], v2[4], v4[4];
        for (int m = 0; m < 4; ++m) {
            tn[m] = 0.5 * (1.0 - std::cos((2 * m + 1) * M_PI / 8.0));
            values((i + tn[m]) * ds, v2[m], v4[m]);
        }
        // monomial coefficients through the four points (Newton divided differences, then
        // expanded)
        for (int f = 0; f < 2; ++f) {
            double d[4];
            for (int m = 0; m < 4; ++m) d[m] = f == 0 ? v2[m] : v4[m];
            for (int lvl = 1; lvl < 4; ++lvl)
                for (int m = 3; m >= lvl; --m) d[m] = (d[m] - d[m - 1]) / (tn[m] - tn[m - lvl]);
            // p(t) = d0 + d1 (t - t0) + d2 (t - t0)(t - t1) + d3 (t - t0)(t - t1)(t - t2)
            double c[4] = {d[3], 0.0, 0.0, 0.0};   // Horner expansion, highest degree first
            int deg = 0;
            for (int m = 2; m >= 0; --m) {
                // c(t) <- c(t) * (t - tn[m]) + d[m]
                double nc[4] = {0.0, 0.0, 0.0, 0.0};
                for (int q = 0; q <= deg; ++q) {
                    nc[q] += c[q] * (-tn[m]);
                    nc[q + 1] += c[q];
                }
                nc[0] += d[m];
                ++deg;
                for (int q = 0; q < 4; ++q) c[q] = nc[q];
            }
            for (int q = 0; q < 4; ++q) t.coef[8 * i + 4 * f + q] = (float)c[q];
        }
    }
    values(smax, t.A2max, t.A4max);
    return cache.emplace(P_clamp, std::move(t)).first->second;
}

// ---------------------------------------------------------------------------------------------
// arena layout
// ---------------------------------------------------------------------------------------------

struct Arena {
    size_t off = 0;
    char *base = nullptr;
    size_t take(size_t bytes) {
        size_t o = (off + 255) & ~(size_t)255;
        off = o + bytes;
        return o;
    }
    template <typename T> T *ptr(size_t o) const { return reinterpret_cast<T *>(base + o); }
};

struct BodyPlan {
    int sim, n, ps, nside;
    size_t oR0, oR1, oF, oOrigin, oFib, oVib, oNw, oNix;
};

struct SimPlan {
    int nx, ny;
    size_t N;
    size_t oH0, oH1, oS0, oS1, oP0, oP1, oSE, oV, oSP, oSPP;
    int tab;     // index into the handle's table list
    int blk0, nblk;
};

struct Plan {
    std::vector<SimPlan> sims;
    std::vector<BodyPlan> bodies;
    std::vector<double> clamps;
    std::vector<size_t> oTab;
    size_t oSims, oBodies, oItems, oIbBlk, oSiteBlk, oT, oStatus, oPartial, oOut, oOutAll, oStage;
    std::vector<WorkItem> items;
    std::vector<int2> ib_blk;
    std::vector<SiteBlock> site_blk;
    int T = 256;
    int max_partial = 1;
    size_t bytes = 0;
};

struct Opt {
    int precision = 0, shift = kDefaultShift, watchdog = 0, chunk = 0, kernel = 0, timing = 0, seg = 0, threads = 0;
    int autotune = 0, grid = 0;
    std::string cache;   // autotune cache file, empty: none
};

Opt read_opt(const lb_options *o) {
    Opt r;
    if (!o) return r;
    r.precision = o->precision;
    r.shift = o->fp16_shift > 0 ? o->fp16_shift : kDefaultShift;
    r.watchdog = o->watchdog_every;
    r.chunk = o->graph_chunk;
    r.kernel = o->kernel;
    r.timing = o->timing;
    r.seg = o->seg_rows;
    r.threads = o->fused_threads;
    r.autotune = o->autotune;
    r.grid = o->grid;
    if (o->autotune_cache) r.cache = o->autotune_cache;
    return r;
}

// centre of a body: the mean of its nodes, or the polygon's centre
void body_centre(const lb_body_desc &b, double &cx, double &cy) {
    cx = b.cx;
    cy = b.cy;
    if (!b.nodes) return;
    cx = cy = 0.0;
    for (int a = 0; a < b.n_nodes; ++a) {
        cx += b.nodes[2 * a];
        cy += b.nodes[2 * a + 1];
    }
    cx /= b.n_nodes;
    cy /= b.n_nodes;
}

double body_extent(const lb_body_desc &b) {
    if (!b.nodes) return b.radius;
    double cx = 0, cy = 0;
    for (int a = 0; a < b.n_nodes; ++a) {
        cx += b.nodes[2 * a];
        cy += b.nodes[2 * a + 1];
    }
    cx /= b.n_nodes;
    cy /= b.n_nodes;
    double r = 0;
    for (int a = 0; a < b.n_nodes; ++a)
        r = std::max(r, std::hypot(b.nodes[2 * a] - cx, b.nodes[2 * a + 1] - cy));
    return r;
}

int validate(const lb_sim_params *sims, int n_sims, const Opt &o) {
    if (!sims || n_sims <= 0) return fail(LB_EINVAL, "need at least one simulation");
    if (o.precision != 0 && o.precision != 1) return fail(LB_EINVAL, "precision must be 0 or 1");
    if (o.shift < 0 || o.shift > 24) return fail(LB_EINVAL, "fp16_shift out of range");
    if (o.kernel != 0 && o.kernel != 1) return fail(LB_EINVAL, "kernel must be 0 or 1");
    if (o.chunk < 0 || (o.chunk & 1)) return fail(LB_EINVAL, "graph_chunk must be even and >= 0");
    if (o.threads != 0 && o.threads != 64 && o.threads != 128 && o.threads != 256)
        return fail(LB_EINVAL, "fused_threads must be 0, 64, 128 or 256");
    if (o.seg < 0) return fail(LB_EINVAL, "seg_rows must be >= 0");
    if (o.grid < 0) return fail(LB_EINVAL, "grid must be >= 0");
    for (int s = 0; s < n_sims; ++s) {
        const lb_sim_params &p = sims[s];
        if (p.nx < 8 || p.ny < 8 || p.nx > 16384 || p.ny > 16384) return fail(LB_EINVAL, "sim %d: lattice size out of range", s);
        if ((long long)p.nx * p.ny > 100000000LL) return fail(LB_EINVAL, "sim %d: more than 1e8 lattice sites", s);
        if (!(p.tau > 0.5)) return fail(LB_EINVAL, "sim %d: tau must exceed 0.5", s);
        if (!(p.D_p >= 0.0) || !(8.0 * p.D_p < 2.0)) return fail(LB_EINVAL, "sim %d: need 0 <= D_p and 8 D_p < 2", s);
        if (!(p.eta_p > 0.0)) return fail(LB_EINVAL, "sim %d: eta_p must be positive", s);
        if (!(p.P_clamp > 0.0 && p.P_clamp < 1.0)) return fail(LB_EINVAL, "sim %d: P_clamp must be in (0, 1)", s);
        if (p.walls < 0 || p.walls > 2) return fail(LB_EINVAL, "sim %d: walls must be 0, 1 or 2", s);
        if (!std::isfinite(p.gx) || !std::isfinite(p.gy)) return fail(LB_EINVAL, "sim %d: gx, gy must be finite", s);
        if (p.n_bodies < 0 || p.n_bodies > kMaxBodies) return fail(LB_EINVAL, "sim %d: n_bodies out of range", s);
        if (p.n_bodies > 0 && !p.bodies) return fail(LB_EINVAL, "sim %d: bodies is NULL", s);
        for (int b = 0; b < p.n_bodies; ++b) {
            const lb_body_desc &d = p.bodies[b];
            if (d.n_nodes < 3 || d.n_nodes > kMaxNodes) return fail(LB_EINVAL, "sim %d body %d: n_nodes out of range", s, b);
            if (!d.nodes && !(d.radius > 0.0)) return fail(LB_EINVAL, "sim %d body %d: radius must be positive", s, b);
            if (d.trap_k != 0.0 && (!(d.trap_w > 0.0) || !(d.trap_t2 >= d.trap_t1) || !std::isfinite(d.trap_k)))
                return fail(LB_EINVAL, "sim %d body %d: trap needs trap_w > 0 and trap_t2 >= trap_t1", s, b);
            double ext = body_extent(d);
            int lim = std::min(p.nx, p.ny);
            if (2 * (int)std::ceil(ext) + 8 > lim)
                return fail(LB_EINVAL, "sim %d body %d: body too large for the lattice", s, b);
            if (p.walls) {
                // every node's kernel footprint (rows floor(y) - 1 .. floor(y) + 2) inside the walls,
                // with one row to spare for the predicted position
                double lo = d.cy - ext, hi = d.cy + ext;
                if (d.nodes) {
                    lo = hi = d.nodes[1];
                    for (int a = 0; a < d.n_nodes; ++a) {
                        lo = std::min(lo, d.nodes[2 * a + 1]);
                        hi = std::max(hi, d.nodes[2 * a + 1]);
                    }
                }
                double lox = d.cx - ext, hix = d.cx + ext;
                if (d.nodes) {
                    lox = hix = d.nodes[0];
                    for (int a = 0; a < d.n_nodes; ++a) {
                        lox = std::min(lox, d.nodes[2 * a]);
                        hix = std::max(hix, d.nodes[2 * a]);
                    }
                }
                if (std::floor(lo) - 2 < 0 || std::floor(hi) + 3 > p.ny - 1 ||
                    (p.walls == 2 && (std::floor(lox) - 2 < 0 || std::floor(hix) + 3 > p.nx - 1)))
                    return fail(LB_EINVAL, "sim %d body %d: a node's kernel footprint reaches a wall", s, b);
            }
        }
        // bodies do not overlap: their bounding circles (centre of the nodes, farthest node) stay
        // apart, measured across the periodic directions
        for (int b = 0; b < p.n_bodies; ++b)
            for (int c = b + 1; c < p.n_bodies; ++c) {
                double xb, yb, xc, yc;
                body_centre(p.bodies[b], xb, yb);
                body_centre(p.bodies[c], xc, yc);
                double dx = std::fabs(xb - xc), dy = std::fabs(yb - yc);
                if (p.walls != 2) {
                    dx = std::fmod(dx, (double)p.nx);
                    dx = std::min(dx, p.nx - dx);
                }
                if (p.walls == 0) {
                    dy = std::fmod(dy, (double)p.ny);
                    dy = std::min(dy, p.ny - dy);
                }
                if (std::hypot(dx, dy) < body_extent(p.bodies[b]) + body_extent(p.bodies[c]))
                    return fail(LB_EINVAL, "sim %d: bodies %d and %d overlap", s, b, c);
            }
    }
    return LB_OK;
}

int pick_threads(const lb_sim_params *sims, int n_sims, const Opt &o) {
    if (o.threads) return o.threads;
    int mx = 0;
    for (int s = 0; s < n_sims; ++s) mx = std::max(mx, sims[s].nx);
    return mx <= 120 ? 128 : 256;
}

Plan make_plan(const lb_sim_params *sims, int n_sims, const Opt &o) {
    Plan pl;
    Arena a;
    pl.T = pick_threads(sims, n_sims, o);
    const size_t hb = o.precision == 1 ? 2 : 4;
    int nblk_sites = 0;
    size_t maxN = 0;
    int total_bodies = 0;
    for (int s = 0; s < n_sims; ++s) total_bodies += sims[s].n_bodies;
    // distinct clamps -> tables
    for (int s = 0; s < n_sims; ++s) {
        double c = sims[s].P_clamp;
        if (std::find(pl.clamps.begin(), pl.clamps.end(), c) == pl.clamps.end()) pl.clamps.push_back(c);
    }
    pl.oSims = a.take(sizeof(SimDev) * n_sims);
    pl.oBodies = a.take(sizeof(BodyDev) * std::max(1, total_bodies));
    for (size_t i = 0; i < pl.clamps.size(); ++i) pl.oTab.push_back(a.take(sizeof(float) * 8 * kStiffSeg));
    for (int s = 0; s < n_sims; ++s) {
        const lb_sim_params &p = sims[s];
        SimPlan sp;
        sp.nx = p.nx;
        sp.ny = p.ny;
        sp.N = (size_t)p.nx * p.ny;
        maxN = std::max(maxN, sp.N);
        sp.oH0 = a.take(9 * sp.N * hb);
        sp.oH1 = a.take(9 * sp.N * hb);
        sp.oS0 = a.take(3 * sp.N * 4);
        sp.oS1 = a.take(3 * sp.N * 4);
        const size_t pb = o.precision == 1 ? 4 : 8;   // polarization: FP32 offsets with FP16 populations
        sp.oP0 = a.take(2 * sp.N * pb);
        sp.oP1 = a.take(2 * sp.N * pb);
        sp.oSE = a.take(4 * sp.N * 4);
        sp.oV = a.take(o.kernel == 1 ? 2 * sp.N * 4 : 0);
        sp.oSP = a.take(o.kernel == 1 ? 3 * sp.N * 4 : 0);
        sp.oSPP = a.take(o.kernel == 1 ? 2 * sp.N * pb : 0);
        sp.tab = (int)(std::find(pl.clamps.begin(), pl.clamps.end(), p.P_clamp) - pl.clamps.begin());
        sp.blk0 = nblk_sites;
        sp.nblk = (int)((sp.N + 255) / 256);
        for (int b = 0; b < sp.nblk; ++b) pl.site_blk.push_back(SiteBlock{s, b * 256});
        nblk_sites += sp.nblk;
        for (int b = 0; b < p.n_bodies; ++b) {
            const lb_body_desc &d = p.bodies[b];
            BodyPlan bp;
            bp.sim = s;
            bp.n = d.n_nodes;
            bp.ps = std::min(2 * (int)std::ceil(body_extent(d)) + 24, std::min(p.nx, p.ny));
            bp.nside = (bp.ps + kPatchTile - 1) / kPatchTile;
            bp.oR0 = a.take(16 * (size_t)bp.n);
            bp.oR1 = a.take(16 * (size_t)bp.n);
            bp.oF = a.take(16 * (size_t)bp.n);
            bp.oOrigin = a.take(8 * sizeof(int));
            bp.oFib = a.take(2 * (size_t)bp.ps * bp.ps * 4);
            bp.oVib = a.take(2 * (size_t)bp.ps * bp.ps * 4);
            bp.oNw = a.take(32 * (size_t)bp.n);
            bp.oNix = a.take(8 * (size_t)bp.n);
            for (int q = 0; q < bp.nside * bp.nside; ++q) pl.ib_blk.push_back(make_int2((int)pl.bodies.size(), q));
            pl.bodies.push_back(bp);
        }
        pl.sims.push_back(sp);
    }
    // fused work items are built in lb_create (they depend on the device); reserve room for
    // the shortest segments any choice may use
    size_t max_items = 0;
    for (int s = 0; s < n_sims; ++s) {
        int W = 64 - 2 * kHalo;   // the narrowest strips any work-group size uses
        max_items += (size_t)((sims[s].nx + W - 1) / W) * (size_t)((sims[s].ny + 3) / 4);
    }
    pl.items.resize(max_items);
    pl.oItems = a.take(sizeof(WorkItem) * pl.items.size());
    pl.oIbBlk = a.take(sizeof(int2) * std::max<size_t>(1, pl.ib_blk.size()));
    pl.oSiteBlk = a.take(sizeof(SiteBlock) * pl.site_blk.size());
    pl.oT = a.take(sizeof(int));
    pl.oStatus = a.take(sizeof(int));
    pl.max_partial = 1024;
    pl.oPartial = a.take(sizeof(double) * 3 * pl.max_partial);
    pl.oOut = a.take(sizeof(double) * 16);
    pl.oOutAll = a.take(sizeof(double) * kBodyOut * std::max(1, total_bodies));
    pl.oStage = a.take(10 * maxN * 4);
    pl.bytes = a.off + 256;
    return pl;
}

// Work items: a lattice no wider than T is one full-width strip (no halo lanes); a wider one is cut
// into strips of T-8 columns and one narrower remainder, so only the remainder's block carries
// idle lanes; segments of about seg rows.  When the last full strip and the remainder, cut into
// two equal strips instead, take no more waves (for 2048 columns at T = 256: 248 + 64 columns in
// 4 + 2 waves, or 156 + 156 in 3 + 3), they are: more of the items then leave a wave idle, and one
// such item on each unit with four work-groups takes a wave off the busiest units.
int strip_waves(int w) { return (w + 2 * kHalo + 63) / 64; }

std::vector<WorkItem> build_items(const std::vector<SimPlan> &sims, int T, int seg) {
    std::vector<WorkItem> items;
    const int W = T - 2 * kHalo;
    for (size_t s = 0; s < sims.size(); ++s) {
        int nx = sims[s].nx, ny = sims[s].ny;
        const bool full = nx <= T;
        int ns = full ? 1 : (nx + W - 1) / W;
        std::vector<int> sx0, sw;   // strip origins and widths
        for (int k = 0; k < ns; ++k) {
            sx0.push_back(full ? 0 : k * W);
            sw.push_back(full ? nx : std::min(nx, (k + 1) * W) - k * W);
        }
        if (!full && ns >= 2) {
            const int rem = sw[ns - 1], wa = (W + rem) / 2, wb = W + rem - wa;
            if (rem < W && strip_waves(wa) + strip_waves(wb) <= strip_waves(W) + strip_waves(rem)) {
                sw[ns - 2] = wa;
                sx0[ns - 1] = sx0[ns - 2] + wa;
                sw[ns - 1] = wb;
            }
        }
        int ng = std::max(1, (ny + seg - 1) / seg);
        for (int g = 0; g < ng; ++g) {
            int y0 = (int)((long)g * ny / ng), y1 = (int)((long)(g + 1) * ny / ng);
            for (int k = 0; k < ns; ++k)
                items.push_back(WorkItem{(int)s, sx0[k], y0, sw[k], y1 - y0, full ? 1 : 0, 0, 0});
        }
    }
    return items;
}

// cost model of one fused launch: work items run in rounds of `slots` resident work-groups and
// an item of seg rows takes seg + 8 row iterations (the pipeline fill)
int model_seg(const std::vector<SimPlan> &sims, int T, int slots) {
    int best = 8;
    double best_cost = 1e300;
    for (int seg = 4; seg <= 128; ++seg) {
        size_t items = build_items(sims, T, seg).size();
        double rounds = std::ceil((double)items / slots);
        double cost = rounds * (seg + 8) + 1e-3 * seg;   // ties: shorter segments
        if (cost < best_cost) {
            best_cost = cost;
            best = seg;
        }
    }
    return best;
}

}  // namespace

struct lb_handle {
    int n_sims = 0;
    Opt opt;
    Plan plan;
    std::vector<lb_sim_params> params;
    std::vector<std::vector<lb_body_desc>> bdesc;
    std::vector<SimDev> hs;
    std::vector<BodyDev> hb;
    std::vector<double> mass0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *arena = nullptr;
    SimDev *d_sims = nullptr;
    BodyDev *d_bodies = nullptr;
    WorkItem *d_items = nullptr;
    int2 *d_ib = nullptr;
    SiteBlock *d_site = nullptr;
    int *d_t = nullptr;
    int *d_status = nullptr;
    double *d_partial = nullptr;
    double *d_out = nullptr;
    double *d_out_all = nullptr;
    float *d_stage = nullptr;
    int64_t t = 0;
    int cur = 0;
    int fused_grid = 0;
    int fused_T = 256;
    int fused_seg = 0;
    bool any_walls = false;   // some simulation has walls: launch the fused variant that handles them
    bool any_pol = false;     // some simulation has a polarization field; if none, P stays 0 and the
                              // fused variant without the P and Ericksen work runs
    int n_items = 0;
    int cus = 1;   // compute units of the device (the fused kernel's first-round order)
    float tuned_ms = 0.f;
    // graph replay: executable graphs of graph_chunk steps and of every power of two below it, each
    // captured from parity 0 (even lengths, so a replay ends at parity 0 again)
    std::vector<std::pair<int, hipGraphExec_t>> graphs;   // (steps, graph), longest first
    // timing
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending_field, pending_ib;
    double field_ms = 0, ib_ms = 0;
    int64_t field_n = 0, ib_n = 0;
    // watchdog
    int *h_status = nullptr;   // pinned
    hipEvent_t ev_wd = nullptr;
    bool wd_pending = false;

    // releases everything the handle created (also when lb_create fails part way); the arena
    // belongs to the caller
    ~lb_handle() {
        if (stream) (void)hipStreamSynchronize(stream);
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
        for (auto &pr : pending_field) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        for (auto &pr : pending_ib) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        for (auto e : ev_pool) (void)hipEventDestroy(e);
        if (ev_wd) (void)hipEventDestroy(ev_wd);
        if (h_status) (void)hipHostFree(h_status);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

int check_status(lb_handle *h) {
    int st = 0;
    HIPCHK(hipMemcpyAsync(&st, h->d_status, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (st & kStatusUnstable) return fail(LB_EUNSTABLE, "watchdog: non-finite or drifting mass");
    if (st & kStatusPatch) return fail(LB_ERANGE, "a body outgrew its force patch (node motion too large)");
    if (st & kStatusWall) return fail(LB_ERANGE, "a node's kernel footprint reached a wall");
    return LB_OK;
}

hipEvent_t pool_event(lb_handle *h) {
    if (!h->ev_pool.empty()) {
        hipEvent_t e = h->ev_pool.back();
        h->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int drain_timing(lb_handle *h) {
    HIPCHK(hipStreamSynchronize(h->stream));
    for (auto &pr : h->pending_field) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
        h->field_ms += ms;
        h->field_n += 1;
        h->ev_pool.push_back(pr.first);
        h->ev_pool.push_back(pr.second);
    }
    for (auto &pr : h->pending_ib) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
        h->ib_ms += ms;
        h->ib_n += 1;
        h->ev_pool.push_back(pr.first);
        h->ev_pool.push_back(pr.second);
    }
    h->pending_field.clear();
    h->pending_ib.clear();
    return LB_OK;
}

// launch one step's kernels (field pass + node update); parity flips
int launch_step(lb_handle *h, bool timed) {
    const bool fp16 = h->opt.precision == 1;
    hipEvent_t a = nullptr, b = nullptr;
    if (timed) {
        a = pool_event(h);
        b = pool_event(h);
        if (!a || !b) return fail(LB_EDEVICE, "hipEventCreate failed");
        HIPCHK(hipEventRecord(a, h->stream));
    }
    if (h->opt.kernel == 0) {
        HIPCHK(launch_fused(h->fused_T, fp16, h->any_walls, h->any_pol, h->fused_grid, h->stream, h->d_sims, h->d_bodies, h->d_items,
                            h->n_items, h->cur, h->d_t, h->cus));
    } else {
        HIPCHK(launch_multipass(fp16, (int)h->plan.site_blk.size(), h->stream, h->d_sims, h->d_bodies, h->d_site,
                                h->cur, h->d_t));
    }
    if (timed) {
        HIPCHK(hipEventRecord(b, h->stream));
        h->pending_field.emplace_back(a, b);
    }
    if (!h->plan.ib_blk.empty()) {
        hipEvent_t c = nullptr, d = nullptr;
        if (timed) {
            c = pool_event(h);
            d = pool_event(h);
            if (!c || !d) return fail(LB_EDEVICE, "hipEventCreate failed");
            HIPCHK(hipEventRecord(c, h->stream));
        }
        HIPCHK(launch_ib(true, (int)h->plan.bodies.size(), (int)h->plan.ib_blk.size(), h->stream, h->d_sims,
                         h->d_bodies, h->d_ib, h->cur, h->d_t, h->d_status));
        if (timed) {
            HIPCHK(hipEventRecord(d, h->stream));
            h->pending_ib.emplace_back(c, d);
        }
    }
    h->cur ^= 1;
    h->t += 1;
    if (timed && h->pending_field.size() >= 256) {
        int rc = drain_timing(h);
        if (rc) return rc;
    }
    return LB_OK;
}

// the work item of work-group b among n (the fused kernel's xcd_remap: each XCD a contiguous run)
int item_of_block(int b, int n) {
    const int q = n >> 3, r = n & 7, x = b & 7, k = b >> 3;
    return x * q + std::min(x, r) + k;
}

// do the periodic intervals [a, a + la) and [b, b + lb) on a ring of n sites intersect? (the
// fused kernel's ring_overlap)
bool ring_overlap_h(int a, int la, int b, int lb, int n) {
    if (la >= n || lb >= n) return true;
    int d = b - a;
    d = d < 0 ? d + n : d;
    if (d < la) return true;
    int e = a - b;
    e = e < 0 ? e + n : e;
    return e < lb;
}

int wrap_h(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// A launch of at most four work-groups per compute unit deals them to the units in turn: work-group
// b runs on unit b mod cus as its (b / cus)-th, so the units from n - 3 cus on hold three.  Items
// that reach a body's force patch are the slowest (their spread-force reads), and a unit with two
// of them finishes last.  Each is moved to the first work-group of its own unit, the three-item
// units first, by swapping it with the item there.  The patches are those of the current step;
// bodies drift by a small fraction of a site per step, so the order holds for long runs, and it
// only ever changes which work-group takes an item, never the item.
int place_body_items(lb_handle *h, std::vector<WorkItem> &items) {
    const int n = (int)items.size(), cus = h->cus;
    if (h->hb.empty() || n <= cus || n > 4 * cus) return LB_OK;
    struct Patch {
        int sim, ox, oy, ps;
    };
    std::vector<Patch> patches;
    for (size_t b = 0; b < h->hb.size(); ++b) {
        int o[2] = {0, 0};
        HIPCHK(hipMemcpy(o, h->hb[b].origin + 4 * h->cur + 2, sizeof o, hipMemcpyDeviceToHost));
        patches.push_back(Patch{h->plan.bodies[b].sim, o[0], o[1], h->plan.bodies[b].ps});
    }
    std::vector<char> slow(n, 0);
    for (int i = 0; i < n; ++i) {
        const WorkItem &wi = items[i];
        const int nx = h->plan.sims[wi.sim].nx, ny = h->plan.sims[wi.sim].ny;
        const int lanes = wi.full ? wi.w : wi.w + 2 * kHalo;
        for (const Patch &p : patches)
            if (p.sim == wi.sim && ring_overlap_h(p.ox, p.ps, wi.full ? 0 : wrap_h(wi.x0 - kHalo, nx), lanes, nx) &&
                ring_overlap_h(p.oy, p.ps, wrap_h(wi.y0 - 2, ny), wi.l + 4, ny))
                slow[i] = 1;
    }
    std::vector<int> of_block(n), block_of(n);   // item index taken by each work-group, and back
    for (int b = 0; b < n; ++b) {
        of_block[b] = item_of_block(b, n);
        block_of[of_block[b]] = b;
    }
    const int light = std::max(0, n - 3 * cus);   // first work-group of the first three-item unit
    auto move = [&](int i, int t) {   // item i to work-group t, the item there to i's work-group
        const int b = block_of[i], j = of_block[t];
        std::swap(of_block[b], of_block[t]);
        block_of[i] = t;
        block_of[j] = b;
    };
    std::vector<char> hasBody(cus, 0);
    int next = 0;
    for (int i = 0; i < n && next < cus; ++i) {
        if (!slow[i]) continue;
        const int t = (light + next++) % cus;   // the first work-groups, three-item units first
        move(i, t);
        hasBody[t] = 1;
    }
    // then the items with an idle wave, one on each four-item unit that runs no body item (as its
    // second work-group), so that no unit runs four items of full waves where this can be avoided;
    // each goes to a unit of its own XCD (work-group b runs on XCD b mod 8, and so do all of a
    // unit's work-groups when cus is a multiple of 8), where its neighbours' rows are in the L2
    int maxw = 0;
    for (const WorkItem &wi : items) maxw = std::max(maxw, wi.full ? (wi.w + 63) / 64 : strip_waves(wi.w));
    std::vector<char> busy(hasBody);   // units that already run a body item or an idle-wave item
    std::vector<char> done(n, 0);
    for (int i = 0; i < n; ++i) {
        const WorkItem &wi = items[i];
        if (slow[i] || wi.full || strip_waves(wi.w) >= maxw) continue;
        const int x = block_of[i] & 7;
        int t = -1;
        for (int c = (cus % 8 == 0 ? x : 0); c < light && cus + c < n; c += (cus % 8 == 0 ? 8 : 1))
            if (!busy[c]) {
                t = c;
                break;
            }
        if (t < 0) continue;
        move(i, cus + t);
        busy[t] = 1;
        done[i] = 1;
    }
    // the XCDs hold unequal numbers of such items and of free four-item units: the rest go to the
    // four-item units still without one, on any XCD
    int c = 0;
    for (int i = 0; i < n; ++i) {
        const WorkItem &wi = items[i];
        if (done[i] || slow[i] || wi.full || strip_waves(wi.w) >= maxw) continue;
        while (c < light && cus + c < n && busy[c]) ++c;
        if (c >= light || cus + c >= n) break;
        move(i, cus + c);
        busy[c] = 1;
    }
    std::vector<WorkItem> placed(n);
    for (int b = 0; b < n; ++b) placed[item_of_block(b, n)] = items[of_block[b]];
    items.swap(placed);
    return LB_OK;
}

// grid: 0 = one work-group per item; > 0 = persistent grid of that many work-groups (a multiple
// of 8, so each XCD keeps a contiguous run of items) looping over the item table
int upload_items(lb_handle *h, int T, int seg, int grid = 0) {
    std::vector<WorkItem> items = build_items(h->plan.sims, T, seg);
    if (items.size() > h->plan.items.size()) return fail(LB_EINVAL, "internal: work-item table overflow");
    if (grid <= 0 || grid >= (int)items.size()) {
        const int rc = place_body_items(h, items);
        if (rc) return rc;
    }
    HIPCHK(hipMemcpyAsync(h->d_items, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->fused_T = T;
    h->fused_seg = seg;
    h->n_items = (int)items.size();
    h->fused_grid = (grid > 0 && grid < h->n_items) ? grid : h->n_items;
    return LB_OK;
}

// ---- autotune cache: one line per tuned key, "lbtune1 <key> <threads> <seg_rows> <grid> <ms>" ----

// FNV-1a over everything the tuned shape depends on: the lattices (sizes, walls, P or not), the
// storage precision, the field kernel, a forced work-group size, and the GPU (model, CUs)
uint64_t tune_key(const lb_handle *h, const std::vector<lb_sim_params> &sims, int dev) {
    uint64_t k = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int b = 0; b < 8; ++b) {
            k ^= (v >> (8 * b)) & 0xffu;
            k *= 1099511628211ull;
        }
    };
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        for (const char *c = prop.gcnArchName; *c; ++c) mix((uint64_t)(unsigned char)*c);
        mix((uint64_t)prop.multiProcessorCount);
    }
    mix((uint64_t)h->opt.precision);
    mix((uint64_t)h->opt.kernel);
    mix((uint64_t)h->opt.threads);
    mix((uint64_t)sims.size());
    for (const auto &p : sims) {
        mix((uint64_t)p.nx);
        mix((uint64_t)p.ny);
        mix((uint64_t)p.walls);
        mix((uint64_t)(p.init_P != nullptr));
    }
    return k;
}

// the cached shape for `key`, if the file holds a well-formed line for it (the last one wins)
bool tune_lookup(const std::string &path, uint64_t key, int &T, int &seg, int &grid, float &ms) {
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    bool found = false;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        unsigned long long k = 0;
        int t = 0, sg = 0, gr = 0;
        float m = 0.f;
        if (std::sscanf(line, "lbtune1 %llx %d %d %d %f", &k, &t, &sg, &gr, &m) == 5 && k == key &&
            (t == 64 || t == 128 || t == 256) && sg >= 1 && sg <= 4096 && gr >= 0) {
            T = t;
            seg = sg;
            grid = gr;
            ms = m;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

// append one line (a single short write, so concurrent writers do not interleave within it)
void tune_store(const std::string &path, uint64_t key, int T, int seg, int grid, float ms) {
    char line[128];
    const int n = std::snprintf(line, sizeof line, "lbtune1 %016llx %d %d %d %.9g\n", (unsigned long long)key, T, seg,
                                grid, (double)ms);
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;
    if (n > 0) std::fwrite(line, 1, (size_t)n, f);
    std::fclose(f);
}

// Work-group size and segment length of the fused kernel.  Default: the cost model with the
// device's compute units and the kernel's occupancy.  With opt.autotune, every candidate pair
// (T, seg) near the model's choices is timed with HIP events on the live state: a launch reads
// buffer `cur` and writes the other one, so repeating it without flipping the parity changes
// nothing (the step counter it advances is restored afterwards).
int choose_fused_config(lb_handle *h) {
    int dev = 0, cus = 256;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    h->cus = std::max(1, cus);
    if (h->opt.kernel != 0) return LB_OK;
    const bool fp16 = h->opt.precision == 1;
    // work-group width: lattices no wider than 64 or 128 run as full-width strips of that many
    // lanes (no halo lanes and no idle waves); wider ones as 248-column strips of 256 lanes
    auto model_T = [&]() {
        if (h->opt.threads) return h->opt.threads;
        int mx = 0;
        for (const auto &sp : h->plan.sims) mx = std::max(mx, sp.nx);
        return mx <= 64 ? 64 : mx <= 128 ? 128 : 256;
    };
    if (!h->opt.autotune) {
        int T = model_T();
        int seg = h->opt.seg ? h->opt.seg : model_seg(h->plan.sims, T, cus * fused_blocks_per_cu(T, fp16, h->any_walls, h->any_pol));
        return upload_items(h, T, seg, h->opt.grid);
    }
    const uint64_t key = tune_key(h, h->params, dev);
    if (!h->opt.cache.empty()) {
        int T = 0, seg = 0, grid = 0;
        float ms = 0.f;
        if (tune_lookup(h->opt.cache, key, T, seg, grid, ms)) {
            h->tuned_ms = ms;
            return upload_items(h, T, seg, grid);
        }
    }
    struct Cand {
        int T, seg, grid;
        bool operator==(const Cand &o) const { return T == o.T && seg == o.seg && grid == o.grid; }
    };
    std::vector<Cand> cand;
    for (int T : {64, 128, 256}) {
        if (h->opt.threads && T != h->opt.threads) continue;
        int slots = cus * fused_blocks_per_cu(T, fp16, h->any_walls, h->any_pol);
        int m = model_seg(h->plan.sims, T, slots);
        for (int seg : {m, std::max(4, m / 2), m * 2, m + 4, std::max(4, m - 4), 64}) {
            for (int grid : {0, (slots / 8) * 8}) {
                Cand c{T, seg, grid};
                if (std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
            }
        }
    }
    int t_saved = 0;
    HIPCHK(hipMemcpy(&t_saved, h->d_t, sizeof(int), hipMemcpyDeviceToHost));
    // the two timing events, released on every return
    struct EventPair {
        hipEvent_t a = nullptr, b = nullptr;
        ~EventPair() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    HIPCHK(hipEventCreate(&ev.a));
    HIPCHK(hipEventCreate(&ev.b));
    hipEvent_t e0 = ev.a, e1 = ev.b;
    // warm the clocks with the first candidate, then time every candidate in two passes and
    // keep each one's best pass (clock ramps and neighbours on the device add noise)
    {
        int rc = upload_items(h, cand.front().T, cand.front().seg, cand.front().grid);
        if (rc) return rc;
        for (int r = 0; r < 30; ++r)
            HIPCHK(launch_fused(cand.front().T, fp16, h->any_walls, h->any_pol, h->fused_grid, h->stream, h->d_sims, h->d_bodies,
                                h->d_items, h->n_items, h->cur, h->d_t, h->cus));
    }
    std::vector<float> tbest(cand.size(), 1e30f);
    for (int pass = 0; pass < 2; ++pass) {
        for (size_t ci = 0; ci < cand.size(); ++ci) {
            const Cand c = cand[ci];
            int rc = upload_items(h, c.T, c.seg, c.grid);
            if (rc) return rc;
            HIPCHK(launch_fused(c.T, fp16, h->any_walls, h->any_pol, h->fused_grid, h->stream, h->d_sims, h->d_bodies, h->d_items,
                                h->n_items, h->cur, h->d_t, h->cus));
            HIPCHK(hipEventRecord(e0, h->stream));
            for (int r = 0; r < 8; ++r)
                HIPCHK(launch_fused(c.T, fp16, h->any_walls, h->any_pol, h->fused_grid, h->stream, h->d_sims, h->d_bodies, h->d_items,
                                    h->n_items, h->cur, h->d_t, h->cus));
            HIPCHK(hipEventRecord(e1, h->stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            tbest[ci] = std::min(tbest[ci], ms / 8.0f);
        }
    }
    size_t bi = 0;
    for (size_t ci = 1; ci < cand.size(); ++ci)
        if (tbest[ci] < tbest[bi]) bi = ci;
    const Cand pick = cand[bi];
    const float best = tbest[bi];
    HIPCHK(hipMemcpy(h->d_t, &t_saved, sizeof(int), hipMemcpyHostToDevice));
    h->tuned_ms = best;
    if (!h->opt.cache.empty()) tune_store(h->opt.cache, key, pick.T, pick.seg, pick.grid, best);
    return upload_items(h, pick.T, pick.seg, pick.grid);
}

int run_watchdog(lb_handle *h) {
    const bool fp16 = h->opt.precision == 1;
    for (int s = 0; s < h->n_sims; ++s) {
        int nb = std::min(h->plan.max_partial, h->plan.sims[s].nblk);
        HIPCHK(launch_sums(fp16, s, nb, h->stream, h->d_sims, h->cur, h->d_partial, h->d_out, h->mass0[s], h->d_status));
    }
    HIPCHK(hipMemcpyAsync(h->h_status, h->d_status, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipEventRecord(h->ev_wd, h->stream));
    h->wd_pending = true;
    return LB_OK;
}

// capture `steps` coupled steps from parity 0 into an executable graph
int build_graph(lb_handle *h, int steps) {
    hipGraph_t g = nullptr;
    int cur0 = h->cur;
    int64_t t0 = h->t;
    h->cur = 0;
    HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    int rc = LB_OK;
    for (int i = 0; i < steps && rc == LB_OK; ++i) rc = launch_step(h, false);
    hipError_t e = hipStreamEndCapture(h->stream, &g);
    h->cur = cur0;
    h->t = t0;
    if (rc != LB_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(LB_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LB_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    h->graphs.emplace_back(steps, x);
    return LB_OK;
}

// the graphs lb_step replays: graph_chunk steps, then every power of two below it down to 2, so a
// run of n steps replays whole chunks and covers the rest with at most log2(chunk) more graphs
int build_graphs(lb_handle *h) {
    if (h->opt.chunk <= 0 || h->opt.timing) return LB_OK;
    int rc = build_graph(h, h->opt.chunk);
    if (rc) return rc;
    int p = 2;
    while (p * 2 < h->opt.chunk) p *= 2;
    for (; p >= 2; p /= 2) {
        if (p == h->opt.chunk) continue;
        rc = build_graph(h, p);
        if (rc) return rc;
    }
    return LB_OK;
}

}  // namespace

namespace lbk {
void set_last_error(const char *msg) { g_err = msg; }
}  // namespace lbk

extern "C" {

const char *lb_last_error(void) { return g_err.c_str(); }

int lb_query_arena_bytes(const lb_sim_params *sims, int32_t n_sims, const lb_options *opt, size_t *bytes) {
    try {
        if (!bytes) return fail(LB_EINVAL, "bytes is NULL");
        Opt o = read_opt(opt);
        int rc = validate(sims, n_sims, o);
        if (rc) return rc;
        *bytes = make_plan(sims, n_sims, o).bytes;
        return LB_OK;
    } catch (const std::bad_alloc &) {
        return fail(LB_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(LB_EINVAL, "unexpected host error");
    }
}

static int create_impl(const lb_sim_params *sims, int n_sims, const lb_options *opt, void *arena, size_t arena_bytes,
                       void *stream, lb_handle **out) {
    if (!out) return fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!arena) return fail(LB_EINVAL, "device_arena is NULL");
    if (((uintptr_t)arena) & 255) return fail(LB_EINVAL, "device_arena must be 256-byte aligned");
    Opt o = read_opt(opt);
    int rc = validate(sims, n_sims, o);
    if (rc) return rc;
    std::unique_ptr<lb_handle> h(new lb_handle());
    h->n_sims = n_sims;
    for (int s = 0; s < n_sims; ++s) h->any_walls = h->any_walls || sims[s].walls != 0;
    h->opt = o;
    h->plan = make_plan(sims, n_sims, o);
    if (arena_bytes < h->plan.bytes)
        return fail(LB_ENOMEM, "arena too small: %zu bytes given, %zu needed", arena_bytes, h->plan.bytes);
    h->arena = static_cast<char *>(arena);
    if (stream) {
        h->stream = static_cast<hipStream_t>(stream);
    } else {
        HIPCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
        h->own_stream = true;
    }
    Arena A;
    A.base = h->arena;
    const Plan &pl = h->plan;
    const bool fp16 = o.precision == 1;
    const float scale = fp16 ? std::ldexp(1.0f, o.shift) : 1.0f;

    // tables
    std::vector<const Table *> tabs;
    for (size_t i = 0; i < pl.clamps.size(); ++i) {
        tabs.push_back(&stiffness_table(pl.clamps[i]));
        HIPCHK(hipMemcpyAsync(A.ptr<float>(pl.oTab[i]), tabs.back()->coef.data(), sizeof(float) * 8 * kStiffSeg,
                              hipMemcpyHostToDevice, h->stream));
    }
    h->d_sims = A.ptr<SimDev>(pl.oSims);
    h->d_bodies = A.ptr<BodyDev>(pl.oBodies);
    h->d_items = A.ptr<WorkItem>(pl.oItems);
    h->d_ib = A.ptr<int2>(pl.oIbBlk);
    h->d_site = A.ptr<SiteBlock>(pl.oSiteBlk);
    h->d_t = A.ptr<int>(pl.oT);
    h->d_status = A.ptr<int>(pl.oStatus);
    h->d_partial = A.ptr<double>(pl.oPartial);
    h->d_out = A.ptr<double>(pl.oOut);
    h->d_out_all = A.ptr<double>(pl.oOutAll);
    h->d_stage = A.ptr<float>(pl.oStage);

    // simulation descriptors and initial fields
    std::vector<float> buf;
    int body_index = 0;
    for (int s = 0; s < n_sims; ++s) {
        const lb_sim_params &p = sims[s];
        const SimPlan &sp = pl.sims[s];
        const size_t N = sp.N;
        SimDev d{};
        d.nx = p.nx;
        d.ny = p.ny;
        d.nb = p.n_bodies;
        d.b0 = body_index;
        d.omega = (float)(1.0 / p.tau);
        d.guo = (float)(1.0 - 0.5 / p.tau);
        d.inv_eta = (float)(1.0 / p.eta_p);
        d.D = (float)p.D_p;
        d.xi = (float)p.xi;
        d.alpha = (float)p.alpha;
        d.beta = (float)p.beta;
        d.kappa = (float)p.kappa;
        d.Gamma = (float)p.Gamma;
        const double K1111 = p.Kx[0], K1122 = p.Kx[1], K2222 = p.Kx[2], K1212 = p.Kx[3];
        const double cA = K1111 - 2 * K1122 - 4 * K1212 + K2222, cB = K1111 - K2222;
        d.cA8 = (float)(cA / 8);
        d.cA2 = (float)(cA / 2);
        d.cB2 = (float)(cB / 2);
        d.s1 = (float)((3 * K1111 + 2 * K1122 + 4 * K1212 + 3 * K2222) / 8);
        d.s2 = (float)((K1111 + 6 * K1122 - 4 * K1212 + K2222) / 8);
        d.s3 = (float)((K1111 - 2 * K1122 + 4 * K1212 + K2222) / 4);
        d.kap4 = (float)(0.25 * p.kappa);
        d.m4D = (float)(-4.0 * p.D_p);
        d.gk = (float)(p.Gamma * p.kappa);
        const Table &tb = *tabs[sp.tab];
        d.smax = (float)(p.P_clamp * p.P_clamp);
        d.inv_ds = (float)(kStiffSeg / (p.P_clamp * p.P_clamp));
        d.A2max = (float)tb.A2max;
        d.A4max = (float)tb.A4max;
        d.scale = scale;
        d.inv_scale = 1.0f / scale;
        d.ericksen = p.ericksen ? 1 : 0;
        d.walls = p.walls;
        d.gx = (float)p.gx;
        d.gy = (float)p.gy;
        d.tab = A.ptr<float>(pl.oTab[sp.tab]);
        d.h[0] = A.ptr<void>(sp.oH0);
        d.h[1] = A.ptr<void>(sp.oH1);
        d.sig[0] = A.ptr<float>(sp.oS0);
        d.sig[1] = A.ptr<float>(sp.oS1);
        d.P[0] = A.ptr<void>(sp.oP0);
        d.P[1] = A.ptr<void>(sp.oP1);
        d.sE = A.ptr<float>(sp.oSE);
        d.v = o.kernel == 1 ? A.ptr<float>(sp.oV) : nullptr;
        d.sps = o.kernel == 1 ? A.ptr<float>(sp.oSP) : nullptr;
        d.spp = o.kernel == 1 ? A.ptr<void>(sp.oSPP) : nullptr;
        // P: with FP16 populations FP32 offsets from the mean of the initial field (rounded to FP32);
        // with FP32 populations the FP64 values themselves (reference 0)
        {
            double m0 = 0.0, m1 = 0.0;
            if (p.init_P && fp16) {
                for (size_t i = 0; i < N; ++i) {
                    m0 += p.init_P[i];
                    m1 += p.init_P[N + i];
                }
                m0 /= (double)N;
                m1 /= (double)N;
            }
            d.pref[0] = (float)m0;
            d.pref[1] = (float)m1;
            const double r0 = d.pref[0], r1 = d.pref[1];
            d.pref_d[0] = r0;
            d.pref_d[1] = r1;
            d.alpha_d = p.alpha;
            d.beta_d = p.beta;
            if (p.init_P)
                for (size_t i = 0; i < 2 * N; ++i) h->any_pol = h->any_pol || p.init_P[i] != 0.0;
            if (fp16) {
                std::vector<float> pb(2 * N, 0.0f);
                HIPCHK(hipMemcpyAsync(d.P[1], pb.data(), 2 * N * 4, hipMemcpyHostToDevice, h->stream));
                if (p.init_P)
                    for (size_t i = 0; i < N; ++i) {
                        pb[i] = (float)(p.init_P[i] - r0);
                        pb[N + i] = (float)(p.init_P[N + i] - r1);
                    }
                HIPCHK(hipMemcpyAsync(d.P[0], pb.data(), 2 * N * 4, hipMemcpyHostToDevice, h->stream));
                HIPCHK(hipStreamSynchronize(h->stream));
            } else {
                std::vector<double> pb(2 * N, 0.0);
                HIPCHK(hipMemcpyAsync(d.P[1], pb.data(), 2 * N * 8, hipMemcpyHostToDevice, h->stream));
                if (p.init_P) std::copy(p.init_P, p.init_P + 2 * N, pb.begin());
                HIPCHK(hipMemcpyAsync(d.P[0], pb.data(), 2 * N * 8, hipMemcpyHostToDevice, h->stream));
                HIPCHK(hipStreamSynchronize(h->stream));
            }
        }
        h->hs.push_back(d);

        buf.assign(3 * N, 0.0f);
        if (p.init_sigma)
            for (size_t i = 0; i < 3 * N; ++i) buf[i] = (float)p.init_sigma[i];
        HIPCHK(hipMemcpyAsync(d.sig[0], buf.data(), 3 * N * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        // populations: the stored array is post-collision of the previous step, pulled by the
        // next step, so slot (x, y) of plane n holds h_n(x + c_n, y + c_n) - w_n
        static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        static const double WQ[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
        static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
        buf.assign(9 * N, 0.0f);
        if (p.init_h) {
            for (int n = 0; n < 9; ++n)
                for (int y = 0; y < p.ny; ++y)
                    for (int x = 0; x < p.nx; ++x) {
                        int xs = x + CX[n], ys = y + CY[n];
                        // beyond a wall the first pull bounces back: this slot is then read as
                        // the opposite direction at (x, y)
                        const bool out = (p.walls && (ys < 0 || ys >= p.ny)) || (p.walls == 2 && (xs < 0 || xs >= p.nx));
                        const int m = out ? OPP[n] : n;
                        if (out) {
                            xs = x;
                            ys = y;
                        }
                        xs = (xs + p.nx) % p.nx;
                        ys = (ys + p.ny) % p.ny;
                        buf[(size_t)n * N + (size_t)y * p.nx + x] =
                            (float)(p.init_h[(size_t)m * N + (size_t)ys * p.nx + xs] - WQ[n]);
                    }
        }
        HIPCHK(hipMemcpyAsync(h->d_stage, buf.data(), 9 * N * 4, hipMemcpyHostToDevice, h->stream));
        HIPCHK(launch_pack(fp16, h->stream, h->d_stage, d.h[0], 9 * N, scale));
        HIPCHK(hipStreamSynchronize(h->stream));

        // bodies
        h->params.push_back(p);
        h->bdesc.emplace_back(p.bodies, p.bodies + p.n_bodies);
        for (int b = 0; b < p.n_bodies; ++b, ++body_index) {
            const lb_body_desc &bd = p.bodies[b];
            const BodyPlan &bp = pl.bodies[body_index];
            BodyDev B{};
            B.sim = s;
            B.n = bd.n_nodes;
            B.ps = bp.ps;
            B.nside = bp.nside;
            B.k = bd.k_spring;
            B.eps = bd.eps_angle;
            B.leq = bd.l_eq;
            B.fx = bd.pull_fx;
            B.fy = bd.pull_fy;
            B.t_on = bd.pull_t_on;
            B.t_off = bd.pull_t_off;
            B.width = bd.pull_width;
            B.trap_k = bd.trap_k;
            B.trap_x0 = bd.trap_x0;
            B.trap_y0 = bd.trap_y0;
            B.trap_dx = bd.trap_dx;
            B.trap_dy = bd.trap_dy;
            B.trap_t1 = bd.trap_t1;
            B.trap_t2 = bd.trap_t2;
            B.trap_w = bd.trap_w;
            B.R[0] = A.ptr<double>(bp.oR0);
            B.R[1] = A.ptr<double>(bp.oR1);
            B.fnode = A.ptr<double>(bp.oF);
            B.origin = A.ptr<int>(bp.oOrigin);
            B.fib = A.ptr<float>(bp.oFib);
            B.vib = A.ptr<float>(bp.oVib);
            B.nw = A.ptr<float>(bp.oNw);
            B.nix = A.ptr<int>(bp.oNix);
            std::vector<double> R(2 * (size_t)bd.n_nodes);
            for (int a = 0; a < bd.n_nodes; ++a) {
                if (bd.nodes) {
                    R[2 * a] = bd.nodes[2 * a];
                    R[2 * a + 1] = bd.nodes[2 * a + 1];
                } else {
                    double ang = 2.0 * M_PI * a / bd.n_nodes;
                    R[2 * a] = bd.cx + bd.radius * std::cos(ang);
                    R[2 * a + 1] = bd.cy + bd.radius * std::sin(ang);
                }
            }
            const int zero_origin[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            HIPCHK(hipMemcpyAsync(B.origin, zero_origin, sizeof zero_origin, hipMemcpyHostToDevice, h->stream));
            HIPCHK(hipMemcpyAsync(B.R[0], R.data(), R.size() * 8, hipMemcpyHostToDevice, h->stream));
            HIPCHK(hipMemcpyAsync(B.R[1], R.data(), R.size() * 8, hipMemcpyHostToDevice, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
            h->hb.push_back(B);
        }
    }
    HIPCHK(hipMemcpyAsync(h->d_sims, h->hs.data(), sizeof(SimDev) * n_sims, hipMemcpyHostToDevice, h->stream));
    if (!h->hb.empty())
        HIPCHK(hipMemcpyAsync(h->d_bodies, h->hb.data(), sizeof(BodyDev) * h->hb.size(), hipMemcpyHostToDevice, h->stream));
    if (!pl.ib_blk.empty())
        HIPCHK(hipMemcpyAsync(h->d_ib, pl.ib_blk.data(), sizeof(int2) * pl.ib_blk.size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->d_site, pl.site_blk.data(), sizeof(SiteBlock) * pl.site_blk.size(), hipMemcpyHostToDevice,
                          h->stream));
    int zero[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(h->d_t, zero, sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->d_status, zero, sizeof(int), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));

    // initial body forces spread onto their patches
    if (!pl.ib_blk.empty())
        HIPCHK(launch_ib(false, (int)pl.bodies.size(), (int)pl.ib_blk.size(), h->stream, h->d_sims, h->d_bodies,
                         h->d_ib, 0, h->d_t, h->d_status));
    // reference mass for the watchdog
    for (int s = 0; s < n_sims; ++s) {
        int nb = std::min(pl.max_partial, pl.sims[s].nblk);
        HIPCHK(launch_sums(fp16, s, nb, h->stream, h->d_sims, 0, h->d_partial, h->d_out, 0.0, h->d_status));
        double m[3];
        HIPCHK(hipMemcpyAsync(m, h->d_out, sizeof m, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        h->mass0.push_back(m[0]);
    }
    // launch shape of the fused kernel; the autotuner runs the kernel, so only now that every
    // body's patch origin and spread force exist
    HIPCHK(hipStreamSynchronize(h->stream));
    rc = choose_fused_config(h.get());
    if (rc) return rc;
    HIPCHK(hipHostMalloc((void **)&h->h_status, sizeof(int), hipHostMallocDefault));
    *h->h_status = 0;
    HIPCHK(hipEventCreateWithFlags(&h->ev_wd, hipEventDisableTiming));
    rc = check_status(h.get());
    if (rc) return rc;
    rc = build_graphs(h.get());
    if (rc) return rc;
    *out = h.release();
    return LB_OK;
}

int lb_create(const lb_sim_params *sims, int32_t n_sims, const lb_options *opt, void *device_arena, size_t arena_bytes,
              void *hip_stream, lb_handle **out) {
    try {
        return create_impl(sims, n_sims, opt, device_arena, arena_bytes, hip_stream, out);
    } catch (const std::bad_alloc &) {
        return fail(LB_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(LB_EINVAL, "unexpected host error");
    }
}

int lb_step(lb_handle *h, int32_t n_steps) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (n_steps < 0) return fail(LB_EINVAL, "n_steps must be >= 0");
    try {
        if (h->wd_pending && hipEventQuery(h->ev_wd) == hipSuccess) {
            h->wd_pending = false;
            if (*h->h_status & kStatusUnstable) return fail(LB_EUNSTABLE, "watchdog: non-finite or drifting mass");
            if (*h->h_status & kStatusPatch) return fail(LB_ERANGE, "a body outgrew its force patch");
            if (*h->h_status & kStatusWall) return fail(LB_ERANGE, "a node's kernel footprint reached a wall");
        }
        const bool use_graph = !h->graphs.empty();
        int done = 0;
        while (done < n_steps) {
            int rc;
            int left = n_steps - done;
            const int wd = h->opt.watchdog;
            const int until_wd = wd > 0 ? (int)(wd - (h->t % wd)) : left;
            const int lim = std::min(left, until_wd);
            const std::pair<int, hipGraphExec_t> *g = nullptr;
            if (use_graph && h->cur == 0)
                for (const auto &c : h->graphs)   // longest first
                    if (c.first <= lim) {
                        g = &c;
                        break;
                    }
            if (g) {
                HIPCHK(hipGraphLaunch(g->second, h->stream));
                h->t += g->first;
                done += g->first;
            } else {
                rc = launch_step(h, h->opt.timing != 0);
                if (rc) return rc;
                done += 1;
            }
            if (wd > 0 && h->t % wd == 0) {
                rc = run_watchdog(h);
                if (rc) return rc;
            }
        }
        HIPCHK(hipGetLastError());
        return LB_OK;
    } catch (...) {
        return fail(LB_EINVAL, "unexpected host error");
    }
}

int lb_sync(lb_handle *h) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    HIPCHK(hipStreamSynchronize(h->stream));
    return check_status(h);
}

int lb_time(lb_handle *h, int64_t *t) {
    if (!h || !t) return fail(LB_EINVAL, "NULL argument");
    *t = h->t;
    return LB_OK;
}

int lb_read_fields(lb_handle *h, int32_t sim, uint32_t mask, double *out, size_t n_out) {
    if (!h || !out) return fail(LB_EINVAL, "NULL argument");
    if (sim < 0 || sim >= h->n_sims) return fail(LB_ERANGE, "sim index out of range");
    if (mask & ~LB_F_ALL) return fail(LB_EINVAL, "unknown field bits");
    try {
        int rc = check_status(h);
        if (rc) return rc;
        const SimPlan &sp = h->plan.sims[sim];
        const size_t N = sp.N;
        int nplanes = 0;
        for (int b = 0; b < 10; ++b) nplanes += (mask >> b) & 1;
        size_t nodes = 0;
        if (mask & LB_F_NODES)
            for (const auto &bd : h->bdesc[sim]) nodes += 2 * (size_t)bd.n_nodes;
        if (n_out < nplanes * N + nodes) return fail(LB_ERANGE, "output buffer too small");
        if (nplanes) {
            HIPCHK(launch_readout(h->opt.precision == 1, sp.nblk, sp.blk0, h->stream, h->d_sims, h->d_bodies, h->d_site,
                                  h->cur, h->d_stage));
            std::vector<float> st(10 * N);
            HIPCHK(hipMemcpyAsync(st.data(), h->d_stage, 10 * N * 4, hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
            size_t o = 0;
            for (int b = 0; b < 10; ++b) {
                if (!((mask >> b) & 1)) continue;
                const float *src = st.data() + (size_t)b * N;
                if (b == 0)
                    for (size_t i = 0; i < N; ++i) out[o + i] = 1.0 + (double)src[i];
                else
                    for (size_t i = 0; i < N; ++i) out[o + i] = (double)src[i];
                o += N;
            }
        }
        if (mask & LB_F_NODES) {
            size_t o = nplanes * N;
            for (int b = 0; b < h->params[sim].n_bodies; ++b) {
                const BodyDev &B = h->hb[h->hs[sim].b0 + b];
                HIPCHK(hipMemcpyAsync(out + o, B.R[h->cur], 16 * (size_t)B.n, hipMemcpyDeviceToHost, h->stream));
                o += 2 * (size_t)B.n;
            }
            HIPCHK(hipStreamSynchronize(h->stream));
        }
        return check_status(h);
    } catch (const std::bad_alloc &) {
        return fail(LB_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(LB_EINVAL, "unexpected host error");
    }
}

static void body_out(const lb_handle *h, const BodyDev &B, const double *r, double *out) {
    const double t = (double)h->t;
    double pf = 1.0;
    if (B.width > 0.0)
        pf = 1.0 / (1.0 + std::exp(-(t - B.t_on) / B.width)) - 1.0 / (1.0 + std::exp(-(t - B.t_off) / B.width));
    double ex = pf * B.fx, ey = pf * B.fy;
    if (B.trap_k != 0.0) {   // k(t) (R_ext(t) - R_com), with R_com = r[2..3]
        auto S = [](double x) { return 1.0 / (1.0 + std::exp(-x)); };
        auto sp = [](double x) { return x > 30.0 ? x + std::log1p(std::exp(-x)) : std::log1p(std::exp(x)); };
        const double w = B.trap_w, T = B.trap_t2 - B.trap_t1;
        const double k = B.trap_k * (S((t - B.trap_t1) / w) - S((t - B.trap_t2) / w));
        const double rho = T > 0.0 ? (w / T) * (sp((t - B.trap_t1) / w) - sp((t - B.trap_t2) / w)) : 0.0;
        ex += k * (B.trap_x0 + B.trap_dx * rho - r[2]);
        ey += k * (B.trap_y0 + B.trap_dy * rho - r[3]);
    }
    out[0] = r[0];
    out[1] = r[1];
    out[2] = ex;
    out[3] = ey;
    out[4] = r[2];
    out[5] = r[3];
    out[6] = r[4];
    out[7] = r[5];
}

// the batched layout adds the area-weighted restoring force after the 8 values above
constexpr int kBodiesOut = 10;

int lb_body_force(lb_handle *h, int32_t sim, int32_t body, double out[8]) {
    if (!h || !out) return fail(LB_EINVAL, "NULL argument");
    if (sim < 0 || sim >= h->n_sims) return fail(LB_ERANGE, "sim index out of range");
    if (body < 0 || body >= h->params[sim].n_bodies) return fail(LB_ERANGE, "body index out of range");
    int rc = check_status(h);
    if (rc) return rc;
    const int bi = h->hs[sim].b0 + body;
    HIPCHK(launch_body_force(h->stream, h->d_sims, h->d_bodies, bi, 1, h->cur, h->d_out_all));
    double r[kBodyOut];
    HIPCHK(hipMemcpyAsync(r, h->d_out_all, sizeof r, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    body_out(h, h->hb[bi], r, out);
    return check_status(h);
}

int lb_body_forces(lb_handle *h, double *out, size_t n_out) {
    if (!h || !out) return fail(LB_EINVAL, "NULL argument");
    const size_t nb = h->hb.size();
    if (n_out < (size_t)kBodiesOut * nb) return fail(LB_ERANGE, "output buffer too small");
    if (nb == 0) return LB_OK;
    int rc = check_status(h);
    if (rc) return rc;
    HIPCHK(launch_body_force(h->stream, h->d_sims, h->d_bodies, 0, (int)nb, h->cur, h->d_out_all));
    std::vector<double> r(kBodyOut * nb);
    HIPCHK(hipMemcpyAsync(r.data(), h->d_out_all, sizeof(double) * kBodyOut * nb, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (size_t b = 0; b < nb; ++b) {
        double *o = out + kBodiesOut * b;
        body_out(h, h->hb[b], r.data() + kBodyOut * b, o);
        o[8] = r[kBodyOut * b + 6];
        o[9] = r[kBodyOut * b + 7];
    }
    return check_status(h);
}

int lb_body_forces_device(lb_handle *h, double *device_out, size_t n_out) {
    if (!h || !device_out) return fail(LB_EINVAL, "NULL argument");
    const size_t nb = h->hb.size();
    if (n_out < (size_t)kBodyOut * nb) return fail(LB_ERANGE, "output buffer too small");
    if (nb == 0) return LB_OK;
    HIPCHK(launch_body_force(h->stream, h->d_sims, h->d_bodies, 0, (int)nb, h->cur, device_out));
    return LB_OK;
}

int lb_state_bytes(lb_handle *h, double *bytes_per_site) {
    if (!h || !bytes_per_site) return fail(LB_EINVAL, "NULL argument");
    const double pop = h->opt.precision == 1 ? 2.0 : 4.0;
    const double pol = h->opt.precision == 1 ? 4.0 : 8.0;
    *bytes_per_site = 2.0 * (9.0 * pop + 3.0 * 4.0 + 2.0 * pol);
    return LB_OK;
}

int lb_stream_copy(const void *src, void *dst, size_t bytes, void *hip_stream) {
    if (!src || !dst) return fail(LB_EINVAL, "NULL argument");
    if ((bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
        return fail(LB_EINVAL, "bytes and both pointers must be multiples of 16");
    HIPCHK(launch_stream_copy(static_cast<hipStream_t>(hip_stream), src, dst, bytes));
    return LB_OK;
}

int lb_conservation(lb_handle *h, int32_t sim, double out[3]) {
    if (!h || !out) return fail(LB_EINVAL, "NULL argument");
    if (sim < 0 || sim >= h->n_sims) return fail(LB_ERANGE, "sim index out of range");
    int rc = check_status(h);
    if (rc) return rc;
    int nb = std::min(h->plan.max_partial, h->plan.sims[sim].nblk);
    HIPCHK(launch_sums(h->opt.precision == 1, sim, nb, h->stream, h->d_sims, h->cur, h->d_partial, h->d_out, 0.0,
                       h->d_status));
    HIPCHK(hipMemcpyAsync(out, h->d_out, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_timing(lb_handle *h, double *field_ms, int64_t *field_n, double *ib_ms, int64_t *ib_n, int32_t reset) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    int rc = drain_timing(h);
    if (rc) return rc;
    if (field_ms) *field_ms = h->field_ms;
    if (field_n) *field_n = h->field_n;
    if (ib_ms) *ib_ms = h->ib_ms;
    if (ib_n) *ib_n = h->ib_n;
    if (reset) {
        h->field_ms = h->ib_ms = 0;
        h->field_n = h->ib_n = 0;
    }
    return LB_OK;
}

int lb_launch_shape(lb_handle *h, int32_t *threads, int32_t *seg_rows, int32_t *n_items, int32_t *grid,
                    double *tuned_ms) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (threads) *threads = h->fused_T;
    if (seg_rows) *seg_rows = h->fused_seg;
    if (n_items) *n_items = h->n_items;
    if (grid) *grid = h->fused_grid;
    if (tuned_ms) *tuned_ms = h->tuned_ms;
    return LB_OK;
}

int lb_destroy(lb_handle *h) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    delete h;   // waits for the stream, then releases what the handle created
    return LB_OK;
}

}  // extern "C"
