// Grid integrals and pointwise helpers.
//
// Integration over the box is a grid sum with weight h^3 (section
// "Introduction"): <a_n|b_n> = h^3 sum_r conj(a_n(r)) b_n(r) per orbital.
// Reductions are deterministic: pass 1 gives each workgroup a fixed
// contiguous range of points; threads accumulate serially, then combine
// across the lanes of a wave with xor shuffles and across waves in LDS in
// wave order; pass 2 adds the per-workgroup partials in a fixed tree order.
// The result depends only on (np, nst), never on timing.
#include "rsg_internal.h"

#include <cmath>

namespace rsg {

namespace {

constexpr int RB = 256;      // threads per reduction workgroup
constexpr int MAXBLK = 2048; // partial sums per orbital

int64_t reduce_blocks(int64_t np) {
    int64_t nb = (np + RB - 1) / RB;
    if (nb > MAXBLK) nb = MAXBLK;
    return nb < 1 ? 1 : nb;
}

int reduce_ol(int64_t nst) {
    int ol = 1;
    while (ol < nst && ol < 64) ol <<= 1;
    return ol;
}

struct RArgs {
    const double2 *a;
    const double2 *b;
    const int32_t *ijk;
    int64_t np, nst, ld, chunk, nstp;
    double h, off;
    int32_t axis;
    double *part;
};

// KIND 0: conj(a) b; 1: |a|^2; 2: x_axis |a|^2.
template <int KIND, int OL>
__global__ void __launch_bounds__(RB) k_reduce_partial(RArgs r) {
    constexpr int PL = RB / OL;
    __shared__ double red[RB / 64][64][2];
    const int t = threadIdx.x;
    const int o = t % OL, pl = t / OL;
    const int64_t s = (int64_t)blockIdx.y * OL + o;
    const bool sok = s < r.nst;
    const int64_t p0 = (int64_t)blockIdx.x * r.chunk;
    const int64_t p1 = min(r.np, p0 + r.chunk);
    double re = 0.0, im = 0.0;
    if (sok) {
        for (int64_t p = p0 + pl; p < p1; p += PL) {
            const double2 va = r.a[p * r.ld + s];
            if (KIND == 0) {
                const double2 vb = r.b[p * r.ld + s];
                re += va.x * vb.x + va.y * vb.y;
                im += va.x * vb.y - va.y * vb.x;
            } else if (KIND == 1) {
                re += va.x * va.x + va.y * va.y;
            } else {
                const double xc = r.h * ((double)r.ijk[3 * p + r.axis] - r.off);
                re += xc * (va.x * va.x + va.y * va.y);
            }
        }
    }
#pragma unroll
    for (int off = OL; off < 64; off <<= 1) {
        re += __shfl_xor(re, off);
        im += __shfl_xor(im, off);
    }
    const int w = t >> 6, l = t & 63;
    red[w][l][0] = re;
    red[w][l][1] = im;
    __syncthreads();
    if (w == 0 && l < OL) {
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < RB / 64; ++k) {  // lane l of each wave holds its wave total
            sr += red[k][l][0];
            si += red[k][l][1];
        }
        const int64_t sg = (int64_t)blockIdx.y * OL + l;
        if (sg < r.nst) {
            r.part[((int64_t)blockIdx.x * r.nstp + sg) * 2 + 0] = sr;
            r.part[((int64_t)blockIdx.x * r.nstp + sg) * 2 + 1] = si;
        }
    }
}

// One workgroup per orbital: sum the nblk partials in a fixed tree order.
__global__ void __launch_bounds__(RB) k_reduce_final(const double *part, int64_t nblk, int64_t nstp,
                                                     int ncomp, double scale, double *out) {
    __shared__ double red[RB][2];
    const int64_t s = blockIdx.x;
    const int t = threadIdx.x;
    double re = 0.0, im = 0.0;
    for (int64_t b = t; b < nblk; b += RB) {
        re += part[(b * nstp + s) * 2 + 0];
        im += part[(b * nstp + s) * 2 + 1];
    }
    red[t][0] = re;
    red[t][1] = im;
    __syncthreads();
    for (int w = RB / 2; w > 0; w >>= 1) {
        if (t < w) {
            red[t][0] += red[t + w][0];
            red[t][1] += red[t + w][1];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[s * ncomp] = scale * red[0][0];
        if (ncomp == 2) out[s * ncomp + 1] = scale * red[0][1];
    }
}

// Adjoint pair sums: per orbital, sum_r sum_{l+m<=3} coef[l][m] conj(mu_l) x nu_m.
struct XArgs {
    const double2 *mu[4];
    const double2 *nu[4];
    double2 coef[4][4];
    const int32_t *ijk;
    int64_t np, nst, ld, chunk, nstp;
    double h, off;
    int32_t axis;
    double *part;
};

template <int OL>
__global__ void __launch_bounds__(RB) k_cross_partial(XArgs r) {
    constexpr int PL = RB / OL;
    __shared__ double red[RB / 64][64][2];
    const int t = threadIdx.x;
    const int o = t % OL, pl = t / OL;
    const int64_t s = (int64_t)blockIdx.y * OL + o;
    const bool sok = s < r.nst;
    const int64_t p0 = (int64_t)blockIdx.x * r.chunk;
    const int64_t p1 = min(r.np, p0 + r.chunk);
    double re = 0.0, im = 0.0;
    if (sok) {
        for (int64_t p = p0 + pl; p < p1; p += PL) {
            const int64_t e = p * r.ld + s;
            const double xc = r.h * ((double)r.ijk[3 * p + r.axis] - r.off);
            double2 nu[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) nu[m] = r.nu[m][e];
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                double wr = 0.0, wi = 0.0;  // w_l = sum_m coef[l][m] nu_m
#pragma unroll
                for (int m = 0; m + l < 4; ++m) {
                    wr += r.coef[l][m].x * nu[m].x - r.coef[l][m].y * nu[m].y;
                    wi += r.coef[l][m].x * nu[m].y + r.coef[l][m].y * nu[m].x;
                }
                const double2 mu = r.mu[l][e];
                re += xc * (mu.x * wr + mu.y * wi);
                im += xc * (mu.x * wi - mu.y * wr);
            }
        }
    }
#pragma unroll
    for (int off = OL; off < 64; off <<= 1) {
        re += __shfl_xor(re, off);
        im += __shfl_xor(im, off);
    }
    const int w = t >> 6, l = t & 63;
    red[w][l][0] = re;
    red[w][l][1] = im;
    __syncthreads();
    if (w == 0 && l < OL) {
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < RB / 64; ++k) {
            sr += red[k][l][0];
            si += red[k][l][1];
        }
        const int64_t sg = (int64_t)blockIdx.y * OL + l;
        if (sg < r.nst) {
            r.part[((int64_t)blockIdx.x * r.nstp + sg) * 2 + 0] = sr;
            r.part[((int64_t)blockIdx.x * r.nstp + sg) * 2 + 1] = si;
        }
    }
}

// g = 2 Re sum_n h^3 S_n for the per-orbital complex sums S_n; added to *dst
// when accumulate != 0.
__global__ void k_two_re_sum(const double *per, int64_t nst, double *dst) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double g = 0.0;
    for (int64_t s = 0; s < nst; ++s) g += per[2 * s];
    *dst = 2.0 * g;
}

struct PwArgs {
    const double2 *src[5];
    double2 coef[5];
    double2 *dst;
    const int32_t *ijk;
    int64_t np, nst, ld;
    double h, off;
    int32_t axis, nterms;
};

// dst = sum_k coef_k src_k (complex coefficients), over the first nst columns.
__global__ void k_lincomb(PwArgs a) {
    const int64_t total = a.np * a.nst;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = g / a.nst, s = g - p * a.nst;
        const int64_t e = p * a.ld + s;
        double re = 0.0, im = 0.0;
        for (int k = 0; k < a.nterms; ++k) {
            const double2 v = a.src[k][e];
            re += a.coef[k].x * v.x - a.coef[k].y * v.y;
            im += a.coef[k].x * v.y + a.coef[k].y * v.x;
        }
        a.dst[e] = make_double2(re, im);
    }
}

// dst = x_axis * src.
__global__ void k_mul_axis(PwArgs a) {
    const int64_t total = a.np * a.nst;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = g / a.nst, s = g - p * a.nst;
        const int64_t e = p * a.ld + s;
        const double xc = a.h * ((double)a.ijk[3 * p + a.axis] - a.off);
        const double2 v = a.src[0][e];
        a.dst[e] = make_double2(xc * v.x, xc * v.y);
    }
}

__global__ void k_accumulate(const double *src, double *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst += *src;
}

unsigned pw_blocks(int64_t total) {
    int64_t nb = (total + 255) / 256;
    if (nb > 65536) nb = 65536;
    return (unsigned)(nb < 1 ? 1 : nb);
}

}  // namespace

size_t reduce_workspace_bytes(const Grid &g, int64_t nst) {
    const int ol = reduce_ol(nst);
    const int64_t nstp = (nst + ol - 1) / ol * ol;
    return (size_t)reduce_blocks(g.np) * (size_t)nstp * 2 * sizeof(double) +
           (size_t)nstp * 2 * sizeof(double) + 256;
}

int launch_reduce(const Grid &g, int kind, int axis, const double2 *a, const double2 *b, int64_t nst,
                  int64_t ld, double *out, void *ws, size_t ws_bytes, hipStream_t s) {
    if (nst == 0) return RSG_OK;
    if (ws_bytes < reduce_workspace_bytes(g, nst)) {
        set_error("reduction workspace too small: %zu < %zu", ws_bytes, reduce_workspace_bytes(g, nst));
        return RSG_ENOMEM;
    }
    const int ol = reduce_ol(nst);
    const int64_t nblk = reduce_blocks(g.np);
    RArgs r;
    r.a = a;
    r.b = b;
    r.ijk = g.ijk;
    r.np = g.np;
    r.nst = nst;
    r.ld = ld;
    r.chunk = (g.np + nblk - 1) / nblk;
    r.nstp = (nst + ol - 1) / ol * ol;
    r.h = g.h;
    r.axis = axis < 0 ? 0 : axis;
    r.off = 0.5 * (double)(g.n[r.axis] - 1);
    r.part = (double *)ws;
    const dim3 grid((unsigned)nblk, (unsigned)(r.nstp / ol));
#define RSG_RED(K)                                                                          \
    switch (ol) {                                                                           \
        case 1: k_reduce_partial<K, 1><<<grid, RB, 0, s>>>(r); break;                      \
        case 2: k_reduce_partial<K, 2><<<grid, RB, 0, s>>>(r); break;                      \
        case 4: k_reduce_partial<K, 4><<<grid, RB, 0, s>>>(r); break;                      \
        case 8: k_reduce_partial<K, 8><<<grid, RB, 0, s>>>(r); break;                      \
        case 16: k_reduce_partial<K, 16><<<grid, RB, 0, s>>>(r); break;                    \
        case 32: k_reduce_partial<K, 32><<<grid, RB, 0, s>>>(r); break;                    \
        default: k_reduce_partial<K, 64><<<grid, RB, 0, s>>>(r); break;                    \
    }
    if (kind == 0) { RSG_RED(0) } else if (kind == 1) { RSG_RED(1) } else { RSG_RED(2) }
#undef RSG_RED
    const double h3 = g.h * g.h * g.h;
    k_reduce_final<<<(unsigned)nst, RB, 0, s>>>(r.part, nblk, r.nstp, kind == 0 ? 2 : 1, h3, out);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

int launch_cross_dots(const Grid &g, int axis, const double2 *const *mu, const double2 *const *nu,
                      const double2 *pair_coef, int64_t nst, int64_t ld, double *out, void *ws,
                      size_t ws_bytes, hipStream_t s) {
    if (ws_bytes < reduce_workspace_bytes(g, nst)) {
        set_error("adjoint reduction workspace too small");
        return RSG_ENOMEM;
    }
    const int ol = reduce_ol(nst);
    const int64_t nblk = reduce_blocks(g.np);
    XArgs r;
    for (int k = 0; k < 4; ++k) {
        r.mu[k] = mu[k];
        r.nu[k] = nu[k];
        for (int m = 0; m < 4; ++m) r.coef[k][m] = pair_coef[4 * k + m];
    }
    r.ijk = g.ijk;
    r.np = g.np;
    r.nst = nst;
    r.ld = ld;
    r.chunk = (g.np + nblk - 1) / nblk;
    r.nstp = (nst + ol - 1) / ol * ol;
    r.h = g.h;
    r.axis = axis;
    r.off = 0.5 * (double)(g.n[axis] - 1);
    r.part = (double *)ws;
    double *per = r.part + nblk * r.nstp * 2;
    const dim3 grid((unsigned)nblk, (unsigned)(r.nstp / ol));
    switch (ol) {
        case 1: k_cross_partial<1><<<grid, RB, 0, s>>>(r); break;
        case 2: k_cross_partial<2><<<grid, RB, 0, s>>>(r); break;
        case 4: k_cross_partial<4><<<grid, RB, 0, s>>>(r); break;
        case 8: k_cross_partial<8><<<grid, RB, 0, s>>>(r); break;
        case 16: k_cross_partial<16><<<grid, RB, 0, s>>>(r); break;
        case 32: k_cross_partial<32><<<grid, RB, 0, s>>>(r); break;
        default: k_cross_partial<64><<<grid, RB, 0, s>>>(r); break;
    }
    const double h3 = g.h * g.h * g.h;
    k_reduce_final<<<(unsigned)nst, RB, 0, s>>>(r.part, nblk, r.nstp, 2, h3, per);
    k_two_re_sum<<<1, 64, 0, s>>>(per, nst, out);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

int launch_axpby_list(const Grid &g, int64_t nst, int64_t ld, int nterms, const double2 *const *src,
                      const double2 *coef, double2 *dst, hipStream_t s) {
    PwArgs a;
    for (int k = 0; k < nterms; ++k) {
        a.src[k] = src[k];
        a.coef[k] = coef[k];
    }
    a.nterms = nterms;
    a.dst = dst;
    a.np = g.np;
    a.nst = nst;
    a.ld = ld;
    k_lincomb<<<pw_blocks(g.np * nst), 256, 0, s>>>(a);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

int launch_mul_axis(const Grid &g, int axis, const double2 *src, double2 *dst, int64_t nst,
                    int64_t ld, hipStream_t s) {
    PwArgs a;
    a.src[0] = src;
    a.dst = dst;
    a.ijk = g.ijk;
    a.np = g.np;
    a.nst = nst;
    a.ld = ld;
    a.h = g.h;
    a.axis = axis;
    a.off = 0.5 * (double)(g.n[axis] - 1);
    k_mul_axis<<<pw_blocks(g.np * nst), 256, 0, s>>>(a);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

int launch_accumulate(const double *src, double *dst, hipStream_t s) {
    k_accumulate<<<1, 64, 0, s>>>(src, dst);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

}  // namespace rsg

// ------------------------------------------------------------------------
// Control field (section "Quantum optimal control": the control is the
// electric-field amplitude, parametrised by its Fourier coefficients).
// ------------------------------------------------------------------------

namespace {

__global__ void k_laser_field(const double *coef, int32_t ncoef, double T, double dt, int64_t step0,
                              int64_t nsteps, double *out) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nsteps) return;
    const double tau = ((double)(step0 + n) + 0.5) * dt;
    double e = 0.0;
    for (int32_t k = 1; k <= ncoef; ++k) e += coef[k - 1] * sin(k * M_PI * tau / T);
    out[n] = e;
}

// grad[k-1] = sum_n sin(k pi tau_n / T) g[n]: one workgroup per coefficient,
// strided partial sums then a fixed tree.
__global__ void __launch_bounds__(256) k_laser_grad(const double *g, int64_t nsteps, double T,
                                                    double dt, double *grad) {
    __shared__ double red[256];
    const int k = blockIdx.x + 1;
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int64_t n = t; n < nsteps; n += 256) {
        const double tau = ((double)n + 0.5) * dt;
        acc += sin(k * M_PI * tau / T) * g[n];
    }
    red[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) grad[k - 1] = red[0];
}

}  // namespace

extern "C" int rsg_laser_field(const double *coef_dev, int32_t ncoef, double T, double dt,
                               int64_t step0, int64_t nsteps, double *out_dev, void *stream) {
    rsg::clear_error();
    RSG_REQUIRE(nsteps >= 0 && ncoef >= 0, RSG_EINVAL, "rsg_laser_field: negative size");
    RSG_REQUIRE(nsteps == 0 || out_dev, RSG_EINVAL, "rsg_laser_field: null output");
    RSG_REQUIRE(ncoef == 0 || coef_dev, RSG_EINVAL, "rsg_laser_field: null coefficients");
    RSG_REQUIRE(T > 0 && dt > 0, RSG_EINVAL, "rsg_laser_field: T and dt must be > 0");
    if (nsteps == 0) return RSG_OK;
    k_laser_field<<<(unsigned)((nsteps + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        coef_dev, ncoef, T, dt, step0, nsteps, out_dev);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

extern "C" int rsg_laser_grad(const double *g_dev, int64_t nsteps, double T, double dt,
                              int32_t ncoef, double *grad_dev, void *stream) {
    rsg::clear_error();
    RSG_REQUIRE(nsteps >= 0 && ncoef >= 0, RSG_EINVAL, "rsg_laser_grad: negative size");
    RSG_REQUIRE((nsteps == 0 || g_dev) && (ncoef == 0 || grad_dev), RSG_EINVAL,
                "rsg_laser_grad: null pointer");
    RSG_REQUIRE(T > 0 && dt > 0, RSG_EINVAL, "rsg_laser_grad: T and dt must be > 0");
    if (ncoef == 0) return RSG_OK;
    k_laser_grad<<<(unsigned)ncoef, 256, 0, (hipStream_t)stream>>>(g_dev, nsteps, T, dt, grad_dev);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}
