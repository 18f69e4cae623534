// Shifted-Hamiltonian linear solves (H + sigma_n) x_n = b_n, one per orbital.
//
// Section "The Sternheimer formulation of linear-response" (eq.
// (sternheimer)): every Sternheimer
// iteration solves such a system with sigma = -eps_n +- omega + i eta, with
// conjugate gradients for a real shift and the quasi-minimal residual method
// (Freund and Nachtigal, Numer. Math. 60, 315 (1991)) for a complex one.
// The Hamiltonian of this library is real symmetric (real potential, real
// projectors, a real field), or complex symmetric once complex-scaled, so
// A = H + sigma is complex symmetric, A^T = A:
// the two-sided Lanczos process of QMR then needs only A, its left vectors
// equal the right ones under the bilinear form u^T v (no conjugation), and
// one H application per iteration suffices.
//
// Design: every per-orbital scalar of the recurrences stays on the device.
// An iteration is the H application plus three passes over the batch, each
// a pointwise update fused with the partial sums that the next scalar step
// needs, and three small kernels (one workgroup per orbital) that add the
// partial sums in a fixed order and advance the recurrences.  Converged
// orbitals are frozen by a flag that every kernel reads first.  The host
// looks at the flags only every few iterations.
#include "rsg_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace rsg {

namespace {

constexpr int SB = 256;       // threads per pass workgroup
constexpr int SMAXBLK = 1024; // partial sums per orbital and quantity
constexpr int NQ = 3;         // quantities summed per pass (at most)

// Per-orbital state of a solve.
struct SolveState {
    double2 sigma;       // shift
    double2 delta;       // QMR: delta_i = v_i^T v_i
    double2 eps;         // QMR: eps_i = p_i^T A p_i; CG: unused
    double2 beta;        // QMR: beta_i = eps_i / delta_i
    double2 eta;         // QMR: eta_{i-1} before the rho step, eta_i after
    double2 cp;          // QMR: coefficient of p_i in p_{i+1}; CG: beta
    double2 alpha;       // CG: step length
    double rho;          // QMR: rho_i = ||v~_i||; CG: r^H r
    double theta, gamma; // QMR: theta_{i-1}, gamma_{i-1}
    double cd;           // QMR: (theta_{i-1} gamma_i)^2
    double inv;          // QMR: 1 / rho_{i+1}
    double bnorm, rnorm;
    double tol;
    int32_t active, iters, status, maxiter;
};

int64_t solve_blocks(int64_t np) {
    int64_t nb = (np + 4 * SB - 1) / (4 * SB);
    return std::max<int64_t>(1, std::min<int64_t>(nb, SMAXBLK));
}

// Points [lo, hi) of block b of nb over np points.
__device__ __forceinline__ void block_range(int64_t np, int b, int nb, int64_t *lo, int64_t *hi) {
    const int64_t per = (np + nb - 1) / nb;
    *lo = std::min<int64_t>(np, (int64_t)b * per);
    *hi = std::min<int64_t>(np, *lo + per);
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// unconjugated product a b and conjugated conj(a) b
__device__ __forceinline__ double2 tdot(double2 a, double2 b) { return cmul(a, b); }
__device__ __forceinline__ double2 hdot(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// Sum K complex values over the workgroup in a fixed order (xor shuffles in
// each wave, then the wave totals in wave order) and store them as this
// block's partials.
template <int K>
__device__ __forceinline__ void store_partials(double2 (&acc)[K], double2 *part) {
    __shared__ double2 wsum[SB / 64][K];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double x = acc[k].x, y = acc[k].y;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            x += __shfl_xor(x, o, 64);
            y += __shfl_xor(y, o, 64);
        }
        if (lane == 0) wsum[wv][k] = make_double2(x, y);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double2 t = wsum[0][k];
            for (int w = 1; w < SB / 64; ++w) t = cadd(t, wsum[w][k]);
            part[k] = t;
        }
    }
}

struct PassArgs {
    const double2 *b;
    double2 *x, *r, *w, *v, *p, *d, *s;
    SolveState *st;
    double2 *part;  // [nst][nblk][NQ]
    int64_t np, ldp;
    int32_t nblk;
};

// ---------------------------------------------------------------- passes
// Grid (nblk, nst): block b of orbital n handles a contiguous point range.

// r = b - w - sigma x (w = H x); CG: p = r; QMR: d = s = 0.  Sums: |r|^2,
// r^T r (QMR) , |b|^2.
template <bool QMR>
__global__ void __launch_bounds__(SB) k_sv_init(PassArgs a) {
    const int n = blockIdx.y, blk = blockIdx.x;
    const double2 sg = a.st[n].sigma;
    const int64_t o = (int64_t)n * a.ldp;
    int64_t lo, hi;
    block_range(a.np, blk, a.nblk, &lo, &hi);
    double2 acc[NQ] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
    for (int64_t i = lo + threadIdx.x; i < hi; i += SB) {
        const double2 bb = a.b[o + i], xx = a.x[o + i], ww = a.w[o + i];
        const double2 sx = cmul(sg, xx);
        const double2 rr = make_double2(bb.x - ww.x - sx.x, bb.y - ww.y - sx.y);
        a.r[o + i] = rr;
        if (QMR) {
            a.d[o + i] = make_double2(0, 0);
            a.s[o + i] = make_double2(0, 0);
        } else {
            a.p[o + i] = rr;
        }
        acc[0].x += cabs2(rr);
        acc[1] = cadd(acc[1], tdot(rr, rr));
        acc[2].x += cabs2(bb);
    }
    store_partials<NQ>(acc, a.part + ((int64_t)n * a.nblk + blk) * NQ);
}

// QMR: v = r / rho_1, p = v.
__global__ void __launch_bounds__(SB) k_sv_qmr_start(PassArgs a) {
    const int n = blockIdx.y, blk = blockIdx.x;
    if (!a.st[n].active) return;
    const double inv = a.st[n].inv;
    const int64_t o = (int64_t)n * a.ldp;
    int64_t lo, hi;
    block_range(a.np, blk, a.nblk, &lo, &hi);
    for (int64_t i = lo + threadIdx.x; i < hi; i += SB) {
        const double2 rr = a.r[o + i];
        const double2 vv = make_double2(rr.x * inv, rr.y * inv);
        a.v[o + i] = vv;
        a.p[o + i] = vv;
    }
}

// Sums over p and w = H p: QMR p^T w, p^T p; CG p^H w, p^H p.
template <bool QMR>
__global__ void __launch_bounds__(SB) k_sv_pw(PassArgs a) {
    const int n = blockIdx.y, blk = blockIdx.x;
    if (!a.st[n].active) return;
    const int64_t o = (int64_t)n * a.ldp;
    int64_t lo, hi;
    block_range(a.np, blk, a.nblk, &lo, &hi);
    double2 acc[2] = {make_double2(0, 0), make_double2(0, 0)};
    for (int64_t i = lo + threadIdx.x; i < hi; i += SB) {
        const double2 pp = a.p[o + i], ww = a.w[o + i];
        if (QMR) {
            acc[0] = cadd(acc[0], tdot(pp, ww));
            acc[1] = cadd(acc[1], tdot(pp, pp));
        } else {
            acc[0] = cadd(acc[0], hdot(pp, ww));
            acc[1].x += cabs2(pp);
        }
    }
    store_partials<2>(acc, a.part + ((int64_t)n * a.nblk + blk) * NQ);
}

// QMR: v~ = w + sigma p - beta v, written over v.  Sums |v~|^2, v~^T v~.
__global__ void __launch_bounds__(SB) k_sv_qmr_vt(PassArgs a) {
    const int n = blockIdx.y, blk = blockIdx.x;
    if (!a.st[n].active) return;
    const double2 sg = a.st[n].sigma, be = a.st[n].beta;
    const int64_t o = (int64_t)n * a.ldp;
    int64_t lo, hi;
    block_range(a.np, blk, a.nblk, &lo, &hi);
    double2 acc[2] = {make_double2(0, 0), make_double2(0, 0)};
    for (int64_t i = lo + threadIdx.x; i < hi; i += SB) {
        const double2 ww = a.w[o + i], pp = a.p[o + i], vv = a.v[o + i];
        const double2 sp = cmul(sg, pp), bv = cmul(be, vv);
        const double2 t = make_double2(ww.x + sp.x - bv.x, ww.y + sp.y - bv.y);
        a.v[o + i] = t;
        acc[0].x += cabs2(t);
        acc[1] = cadd(acc[1], tdot(t, t));
    }
    store_partials<2>(acc, a.part + ((int64_t)n * a.nblk + blk) * NQ);
}

// QMR: d = eta p + cd d; s = eta (w + sigma p) + cd s; x += d; r -= s;
// v = v~ / rho_{i+1}; p = v - cp p.  Sum |r|^2.
__global__ void __launch_bounds__(SB) k_sv_qmr_update(PassArgs a) {
    const int n = blockIdx.y, blk = blockIdx.x;
    if (!a.st[n].active) return;
    const SolveState &q = a.st[n];
    const double2 sg = q.sigma, et = q.eta, cp = q.cp;
    const double cd = q.cd, inv = q.inv;
    const int64_t o = (int64_t)n * a.ldp;
    int64_t lo, hi;
    block_range(a.np, blk, a.nblk, &lo, &hi);
    double2 acc[1] = {make_double2(0, 0)};
    for (int64_t i = lo + threadIdx.x; i < hi; i += SB) {
        const double2 pp = a.p[o + i], ww = a.w[o + i], vt = a.v[o + i];
        double2 dd = a.d[o + i], ss = a.s[o + i], xx = a.x[o + i], rr = a.r[o + i];
        const double2 ep = cmul(et, pp);
        const double2 ap = cadd(ww, cmul(sg, pp));
        const double2 ea = cmul(et, ap);
        dd = make_double2(ep.x + cd * dd.x, ep.y + cd * dd.y);
        ss = make_double2(ea.x + cd * ss.x, ea.y + cd * ss.y);
        xx = cadd(xx, dd);
        rr = make_double2(rr.x - ss.x, rr.y - ss.y);
        const double2 vn = make_double2(vt.x * inv, vt.y * inv);
        const double2 cpp = cmul(cp, pp);
        a.d[o + i] = dd;
        a.s[o + i] = ss;
        a.x[o + i] = xx;
        a.r[o + i] = rr;
        a.v[o + i] = vn;
        a.p[o + i] = make_double2(vn.x - cpp.x, vn.y - cpp.y);
        acc[0].x += cabs2(rr);
    }
    store_partials<1>(acc, a.part + ((int64_t)n * a.nblk + blk) * NQ);
}

// CG: x += alpha p; r -= alpha (w + sigma p).  Sum |r|^2.
__global__ void __launch_bounds__(SB) k_sv_cg_update(PassArgs a) {
    const int n = blockIdx.y, blk = blockIdx.x;
    if (!a.st[n].active) return;
    const double2 sg = a.st[n].sigma, al = a.st[n].alpha;
    const int64_t o = (int64_t)n * a.ldp;
    int64_t lo, hi;
    block_range(a.np, blk, a.nblk, &lo, &hi);
    double2 acc[1] = {make_double2(0, 0)};
    for (int64_t i = lo + threadIdx.x; i < hi; i += SB) {
        const double2 pp = a.p[o + i], ww = a.w[o + i];
        double2 xx = a.x[o + i], rr = a.r[o + i];
        const double2 ap = cadd(ww, cmul(sg, pp));
        xx = cadd(xx, cmul(al, pp));
        const double2 aa = cmul(al, ap);
        rr = make_double2(rr.x - aa.x, rr.y - aa.y);
        a.x[o + i] = xx;
        a.r[o + i] = rr;
        acc[0].x += cabs2(rr);
    }
    store_partials<1>(acc, a.part + ((int64_t)n * a.nblk + blk) * NQ);
}

// CG: p = r + beta p.
__global__ void __launch_bounds__(SB) k_sv_cg_dir(PassArgs a) {
    const int n = blockIdx.y, blk = blockIdx.x;
    if (!a.st[n].active) return;
    const double2 be = a.st[n].cp;
    const int64_t o = (int64_t)n * a.ldp;
    int64_t lo, hi;
    block_range(a.np, blk, a.nblk, &lo, &hi);
    for (int64_t i = lo + threadIdx.x; i < hi; i += SB) {
        const double2 rr = a.r[o + i], pp = a.p[o + i];
        const double2 bp = cmul(be, pp);
        a.p[o + i] = make_double2(rr.x + bp.x, rr.y + bp.y);
    }
}

// ---------------------------------------------------------------- scalars
// One workgroup per orbital: the K partial sums of the orbital's nblk
// blocks, added in a fixed order, then one thread advances the recurrence.

enum ScalStep { SC_INIT_QMR, SC_INIT_CG, SC_EPS, SC_RHO, SC_RES_QMR, SC_ALPHA, SC_RES_CG };

template <int K>
__device__ __forceinline__ void sum_partials(const double2 *part, int nblk, double2 (&out)[K]) {
    __shared__ double2 red[SB][K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double2 t = make_double2(0, 0);
        for (int b = threadIdx.x; b < nblk; b += SB) t = cadd(t, part[(int64_t)b * NQ + k]);
        red[threadIdx.x][k] = t;
    }
    __syncthreads();
    for (int w = SB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < K; ++k) red[threadIdx.x][k] = cadd(red[threadIdx.x][k], red[threadIdx.x + w][k]);
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = red[0][k];
}

// Breakdown tests.  delta = v^T v of a unit-norm Lanczos vector lies in
// [0, 1] in modulus; below DELTA_MIN the bilinear form has (nearly)
// vanished and the recurrence cannot continue.  Other divisors only need
// to be nonzero.
constexpr double TINY = 1e-290;
constexpr double DELTA_MIN = 1e-13;

template <int STEP>
__global__ void __launch_bounds__(SB) k_sv_scal(SolveState *st, const double2 *part, int nblk) {
    const int n = blockIdx.x;
    SolveState &q = st[n];
    if (STEP != SC_INIT_QMR && STEP != SC_INIT_CG && !q.active) return;
    double2 s[NQ];
    sum_partials<NQ>(part + (int64_t)n * nblk * NQ, nblk, s);
    if (threadIdx.x != 0) return;
    if (STEP == SC_INIT_QMR || STEP == SC_INIT_CG) {
        q.bnorm = std::sqrt(s[2].x);
        q.rnorm = std::sqrt(s[0].x);
        q.iters = 0;
        q.status = 0;
        const double target = q.tol * (q.bnorm > 0 ? q.bnorm : 1.0);
        q.active = q.rnorm > target && q.maxiter > 0;
        if (!q.active) {
            q.status = q.rnorm > target ? 1 : 0;
            return;
        }
        if (STEP == SC_INIT_QMR) {
            const double rho = q.rnorm;
            q.rho = rho;
            q.inv = 1.0 / rho;
            q.delta = make_double2(s[1].x / (rho * rho), s[1].y / (rho * rho));
            q.gamma = 1.0;
            q.theta = 0.0;
            q.eta = make_double2(-1.0, 0.0);
            if (std::sqrt(cabs2(q.delta)) < DELTA_MIN) {
                q.active = 0;
                q.status = 2;
            }
        } else {
            q.rho = s[0].x;  // r^H r
        }
    } else if (STEP == SC_EPS) {
        // eps_i = p^T (H + sigma) p, beta_i = eps_i / delta_i
        const double2 e = cadd(s[0], cmul(q.sigma, s[1]));
        q.eps = e;
        if (std::sqrt(cabs2(e)) < TINY) {
            q.active = 0;
            q.status = 2;
            return;
        }
        q.beta = cdiv(e, q.delta);
    } else if (STEP == SC_RHO) {
        // rho_{i+1}, theta_i, gamma_i, eta_i and the update coefficients
        const double rho1 = std::sqrt(s[0].x);
        const double babs = std::sqrt(cabs2(q.beta));
        const double th = rho1 / (q.gamma * babs);
        const double ga = 1.0 / std::sqrt(1.0 + th * th);
        // eta_i = -eta_{i-1} rho_i gamma_i^2 / (beta_i gamma_{i-1}^2)
        const double f = q.rho * ga * ga / (q.gamma * q.gamma);
        const double2 num = make_double2(-q.eta.x * f, -q.eta.y * f);
        q.eta = cdiv(num, q.beta);
        q.cd = (q.theta * ga) * (q.theta * ga);
        q.theta = th;
        q.gamma = ga;
        if (rho1 > 0) {
            q.inv = 1.0 / rho1;
            const double2 dl = make_double2(s[1].x / (rho1 * rho1), s[1].y / (rho1 * rho1));
            // p_{i+1} = v_{i+1} - (rho_{i+1} delta_{i+1} / eps_i) p_i
            q.cp = cdiv(make_double2(rho1 * dl.x, rho1 * dl.y), q.eps);
            q.delta = dl;
        } else {
            // the Krylov space is exhausted: this update is the last
            q.inv = 0.0;
            q.cp = make_double2(0, 0);
            q.delta = make_double2(0, 0);
        }
        q.rho = rho1;
    } else if (STEP == SC_RES_QMR || STEP == SC_RES_CG) {
        q.rnorm = std::sqrt(s[0].x);
        q.iters += 1;
        const double target = q.tol * (q.bnorm > 0 ? q.bnorm : 1.0);
        if (q.rnorm <= target) {
            q.active = 0;
            q.status = 0;
        } else if (STEP == SC_RES_QMR && (q.rho <= 0 || std::sqrt(cabs2(q.delta)) < DELTA_MIN)) {
            q.active = 0;
            q.status = 2;
        } else if (q.iters >= q.maxiter) {
            q.active = 0;
            q.status = 1;
        }
        if (STEP == SC_RES_CG && q.active) {
            // beta = r'^H r' / r^H r, kept in cp for the direction update
            const double rn2 = s[0].x;
            q.cp = make_double2(rn2 / q.rho, 0.0);
            q.rho = rn2;
        }
    } else if (STEP == SC_ALPHA) {
        // alpha = r^H r / p^H (H + sigma) p (real for a real shift)
        const double pap = s[0].x + q.sigma.x * s[1].x;
        if (std::fabs(pap) < TINY) {
            q.active = 0;
            q.status = 2;
            return;
        }
        q.alpha = make_double2(q.rho / pap, 0.0);
    }
}

}  // namespace

}  // namespace rsg

using namespace rsg;

extern "C" size_t rsg_solve_workspace_bytes(rsg_ham_t H, int32_t method, int64_t nst, int64_t ldp) {
    if (!H || nst < 0 || ldp < 1) return 0;
    const int nb = method == RSG_SOLVE_QMR ? 6 : 3;
    const int64_t nblk = solve_blocks(H->g->np);
    return nb * rounded(batch_bytes(nst, ldp, 16)) + rounded(kb_workspace_bytes(*H, nst)) +
           rounded(sizeof(double2) * NQ * nblk * std::max<int64_t>(nst, 1)) +
           rounded(sizeof(SolveState) * std::max<int64_t>(nst, 1)) + 256;
}

extern "C" int rsg_shifted_solve(rsg_ham_t H, const double *shift, const void *b, void *x, int64_t nst,
                                 int64_t ldp, int32_t method, double tol, int32_t maxiter, int32_t check_every,
                                 int32_t *iters, double *rel_res, int32_t *status, void *ws, size_t ws_bytes,
                                 void *stream) {
    clear_error();
    int rc = check_batch(H, b, nst, ldp, "rsg_shifted_solve");
    if (rc) return rc;
    rc = check_batch(H, x, nst, ldp, "rsg_shifted_solve");
    if (rc) return rc;
    RSG_REQUIRE(method == RSG_SOLVE_CG || method == RSG_SOLVE_QMR, RSG_EINVAL,
                "rsg_shifted_solve: unknown method %d", method);
    RSG_REQUIRE(nst >= 1 && nst <= 65535, RSG_ESHAPE, "rsg_shifted_solve: need 1 <= nst <= 65535");
    RSG_REQUIRE(shift, RSG_EINVAL, "rsg_shifted_solve: null shift");
    RSG_REQUIRE(tol >= 0 && std::isfinite(tol) && maxiter >= 0 && check_every >= 1, RSG_EINVAL,
                "rsg_shifted_solve: need tol >= 0, maxiter >= 0, check_every >= 1");
    RSG_REQUIRE(method == RSG_SOLVE_QMR || !H->complex_scaled(), RSG_EINVAL,
                "rsg_shifted_solve: conjugate gradients need a Hermitian Hamiltonian (no complex scaling)");
    for (int64_t n = 0; n < nst; ++n) {
        RSG_REQUIRE(std::isfinite(shift[2 * n]) && std::isfinite(shift[2 * n + 1]), RSG_EINVAL,
                    "rsg_shifted_solve: shift %lld is not finite", (long long)n);
        RSG_REQUIRE(method == RSG_SOLVE_QMR || shift[2 * n + 1] == 0.0, RSG_EINVAL,
                    "rsg_shifted_solve: conjugate gradients need real shifts (orbital %lld)", (long long)n);
    }
    const size_t bytes = batch_bytes(nst, ldp, 16);
    const char *bp = static_cast<const char *>(b), *xp = static_cast<const char *>(x);
    RSG_REQUIRE(bp + bytes <= xp || xp + bytes <= bp, RSG_EINVAL, "rsg_shifted_solve: b and x overlap");
    const bool qmr = method == RSG_SOLVE_QMR;
    const int64_t nblk = solve_blocks(H->g->np);
    Carve c(ws, ws_bytes);
    PassArgs a;
    a.b = static_cast<const double2 *>(b);
    a.x = static_cast<double2 *>(x);
    a.w = static_cast<double2 *>(c.take(bytes));
    a.r = static_cast<double2 *>(c.take(bytes));
    a.p = static_cast<double2 *>(c.take(bytes));
    a.v = qmr ? static_cast<double2 *>(c.take(bytes)) : nullptr;
    a.d = qmr ? static_cast<double2 *>(c.take(bytes)) : nullptr;
    a.s = qmr ? static_cast<double2 *>(c.take(bytes)) : nullptr;
    void *D = c.take(kb_workspace_bytes(*H, nst));
    a.part = static_cast<double2 *>(c.take(sizeof(double2) * NQ * nblk * nst));
    a.st = static_cast<SolveState *>(c.take(sizeof(SolveState) * nst));
    RSG_REQUIRE(c.ok, RSG_ENOMEM, "rsg_shifted_solve: workspace too small (%zu < %zu bytes)", ws_bytes,
                rsg_solve_workspace_bytes(H, method, nst, ldp));
    a.np = H->g->np;
    a.ldp = ldp;
    a.nblk = (int32_t)nblk;
    hipStream_t s = (hipStream_t)stream;
    return guarded([&]() -> int {
        std::vector<SolveState> hs(nst);
        for (int64_t n = 0; n < nst; ++n) {
            SolveState q{};
            q.sigma = make_double2(shift[2 * n], shift[2 * n + 1]);
            q.tol = tol;
            q.maxiter = maxiter;
            hs[n] = q;
        }
        RSG_CHECK_HIP(hipMemcpyAsync(a.st, hs.data(), sizeof(SolveState) * nst, hipMemcpyHostToDevice, s));
        const dim3 pg((unsigned)nblk, (unsigned)nst);
        const unsigned on = (unsigned)nst;
        int r;
        // r0 = b - (H + sigma) x0
        if ((r = hpsi_impl(*H, a.x, a.w, nst, ldp, 0.0, nullptr, D, s))) return r;
        if (qmr) {
            k_sv_init<true><<<pg, SB, 0, s>>>(a);
            k_sv_scal<SC_INIT_QMR><<<on, SB, 0, s>>>(a.st, a.part, a.nblk);
            k_sv_qmr_start<<<pg, SB, 0, s>>>(a);
        } else {
            k_sv_init<false><<<pg, SB, 0, s>>>(a);
            k_sv_scal<SC_INIT_CG><<<on, SB, 0, s>>>(a.st, a.part, a.nblk);
        }
        RSG_CHECK_HIP(hipGetLastError());
        for (int it = 0; it < maxiter; ++it) {
            if (it % check_every == 0) {
                RSG_CHECK_HIP(hipMemcpyAsync(hs.data(), a.st, sizeof(SolveState) * nst, hipMemcpyDeviceToHost, s));
                RSG_CHECK_HIP(hipStreamSynchronize(s));
                bool any = false;
                for (int64_t n = 0; n < nst && !any; ++n) any = hs[n].active != 0;
                if (!any) break;
            }
            if ((r = hpsi_impl(*H, a.p, a.w, nst, ldp, 0.0, nullptr, D, s))) return r;
            if (qmr) {
                k_sv_pw<true><<<pg, SB, 0, s>>>(a);
                k_sv_scal<SC_EPS><<<on, SB, 0, s>>>(a.st, a.part, a.nblk);
                k_sv_qmr_vt<<<pg, SB, 0, s>>>(a);
                k_sv_scal<SC_RHO><<<on, SB, 0, s>>>(a.st, a.part, a.nblk);
                k_sv_qmr_update<<<pg, SB, 0, s>>>(a);
                k_sv_scal<SC_RES_QMR><<<on, SB, 0, s>>>(a.st, a.part, a.nblk);
            } else {
                k_sv_pw<false><<<pg, SB, 0, s>>>(a);
                k_sv_scal<SC_ALPHA><<<on, SB, 0, s>>>(a.st, a.part, a.nblk);
                k_sv_cg_update<<<pg, SB, 0, s>>>(a);
                k_sv_scal<SC_RES_CG><<<on, SB, 0, s>>>(a.st, a.part, a.nblk);
                k_sv_cg_dir<<<pg, SB, 0, s>>>(a);
            }
            RSG_CHECK_HIP(hipGetLastError());
        }
        RSG_CHECK_HIP(hipMemcpyAsync(hs.data(), a.st, sizeof(SolveState) * nst, hipMemcpyDeviceToHost, s));
        RSG_CHECK_HIP(hipStreamSynchronize(s));
        for (int64_t n = 0; n < nst; ++n) {
            const SolveState &q = hs[n];
            if (iters) iters[n] = q.iters;
            if (rel_res) rel_res[n] = q.rnorm / (q.bnorm > 0 ? q.bnorm : 1.0);
            if (status) status[n] = q.active ? 1 : q.status;
        }
        return RSG_OK;
    });
}
