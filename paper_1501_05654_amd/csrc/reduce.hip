// Grid integrals and pointwise helpers.
//
// Integration over the box is a grid sum with weight h^3 (section
// "Introduction"): <a_n|b_n> = h^3 sum_r conj(a_n(r)) b_n(r) per orbital.
// Reductions are deterministic: pass 1 gives each workgroup a fixed
// contiguous range of points of one orbital (orbital-major batches: the
// range is contiguous in memory); threads accumulate serially, then combine
// across the lanes of a wave with xor shuffles and across waves in LDS in
// wave order; pass 2 adds the per-workgroup partials in a fixed tree order.
// The result depends only on (np, nst), never on timing.
#include "rsg_internal.h"

#include <algorithm>
#include <cmath>

namespace rsg {

namespace {

constexpr int RB = 256;      // threads per reduction workgroup
constexpr int MAXBLK = 1024; // partial sums per orbital

int64_t reduce_blocks(int64_t np) {
    int64_t nb = (np + 4 * RB - 1) / (4 * RB);
    if (nb > MAXBLK) nb = MAXBLK;
    return nb < 1 ? 1 : nb;
}

// Sum (re, im) over the workgroup: xor shuffles within each wave, then the
// wave totals in wave order.  Lane 0 of wave 0 gets the result.
__device__ __forceinline__ void block_sum(double &re, double &im, double (*red)[2]) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        re += __shfl_xor(re, off);
        im += __shfl_xor(im, off);
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
        red[w][0] = re;
        red[w][1] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        re = 0.0;
        im = 0.0;
        for (int k = 0; k < RB / 64; ++k) {
            re += red[k][0];
            im += red[k][1];
        }
    }
}

struct RArgs {
    const double2 *a;
    const double2 *b;
    const int32_t *ijk;
    int64_t np, nst, ldp, chunk;
    double h, off;
    int32_t axis;
    double *part;
};

// KIND 0: conj(a) b; 1: |a|^2; 2: x_axis |a|^2; 3: a b (no conjugation, the
// bilinear form of complex scaling).  blockIdx.x = point chunk,
// blockIdx.y = orbital.
template <int KIND>
__global__ void __launch_bounds__(RB) k_reduce_partial(RArgs r) {
    __shared__ double red[RB / 64][2];
    const int64_t n = blockIdx.y;
    const int64_t p0 = (int64_t)blockIdx.x * r.chunk;
    const int64_t p1 = min(r.np, p0 + r.chunk);
    const double2 *a = r.a + n * r.ldp;
    const double2 *b = (KIND == 0 || KIND == 3) ? r.b + n * r.ldp : nullptr;
    double re = 0.0, im = 0.0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += RB) {
        const double2 va = a[p];
        if (KIND == 0) {
            const double2 vb = b[p];
            re += va.x * vb.x + va.y * vb.y;
            im += va.x * vb.y - va.y * vb.x;
        } else if (KIND == 3) {
            const double2 vb = b[p];
            re += va.x * vb.x - va.y * vb.y;
            im += va.x * vb.y + va.y * vb.x;
        } else if (KIND == 1) {
            re += va.x * va.x + va.y * va.y;
        } else {
            const int32_t c = r.ijk[3 * p + r.axis];  // -1: dead slot of a row-aligned grid
            const double xc = c < 0 ? 0.0 : r.h * ((double)c - r.off);
            re += xc * (va.x * va.x + va.y * va.y);
        }
    }
    block_sum(re, im, red);
    if (threadIdx.x == 0) {
        r.part[((int64_t)blockIdx.x * r.nst + n) * 2 + 0] = re;
        r.part[((int64_t)blockIdx.x * r.nst + n) * 2 + 1] = im;
    }
}

// One workgroup per orbital: sum the nblk partials in a fixed tree order.
__global__ void __launch_bounds__(RB) k_reduce_final(const double *part, int64_t nblk, int64_t nst,
                                                     int ncomp, double scale, double *out) {
    __shared__ double red[RB][2];
    const int64_t s = blockIdx.x;
    const int t = threadIdx.x;
    double re = 0.0, im = 0.0;
    for (int64_t b = t; b < nblk; b += RB) {
        re += part[(b * nst + s) * 2 + 0];
        im += part[(b * nst + s) * 2 + 1];
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

// g = 2 Re sum_k a_k h3 sum_b P[k][b]: one workgroup, strided partial sums
// then a fixed tree per stage.
__global__ void __launch_bounds__(RB) k_pair_final(const double2 *P, int64_t nb, double2 a0, double2 a1,
                                                   double2 a2, double2 a3, double h3, double *g) {
    __shared__ double red[RB][2];
    const int t = threadIdx.x;
    const double2 a[4] = {a0, a1, a2, a3};
    double acc = 0.0;
    for (int k = 0; k < 4; ++k) {
        double re = 0.0, im = 0.0;
        for (int64_t b = t; b < nb; b += RB) {
            re += P[(int64_t)k * nb + b].x;
            im += P[(int64_t)k * nb + b].y;
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
        if (t == 0) acc += a[k].x * red[0][0] - a[k].y * red[0][1];  // Re(a_k S_k)
        __syncthreads();
    }
    if (t == 0) *g = 2.0 * h3 * acc;
}

struct PwArgs {
    const double2 *src[1];
    double2 *dst;
    const int32_t *ijk;
    int64_t np, nst, ldp;
    double h, off;
    int32_t axis;
};

// dst = x_axis * src.
__global__ void k_mul_axis(PwArgs a) {
    const int64_t base = (int64_t)blockIdx.y * a.ldp;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.np;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = base + p;
        const int32_t c = a.ijk[3 * p + a.axis];  // -1: dead slot of a row-aligned grid
        const double xc = c < 0 ? 0.0 : a.h * ((double)c - a.off);
        const double2 v = a.src[0][e];
        a.dst[e] = make_double2(xc * v.x, xc * v.y);
    }
}

__global__ void k_accumulate(const double *src, double *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst += *src;
}

dim3 pw_grid(int64_t np, int64_t nst) {
    int64_t nb = (np + 255) / 256;
    const int64_t cap = std::max<int64_t>(1, 8192 / std::max<int64_t>(nst, 1));
    if (nb > cap) nb = cap;
    return dim3((unsigned)(nb < 1 ? 1 : nb), (unsigned)nst);
}

}  // namespace

size_t reduce_workspace_bytes(const Grid &g, int64_t nst) {
    return (size_t)reduce_blocks(g.np) * (size_t)std::max<int64_t>(nst, 1) * 2 * sizeof(double) +
           (size_t)std::max<int64_t>(nst, 1) * 2 * sizeof(double) + 256;
}

int launch_reduce(const Grid &g, int kind, int axis, const double2 *a, const double2 *b, int64_t nst,
                  int64_t ldp, double *out, void *ws, size_t ws_bytes, hipStream_t s) {
    if (nst == 0) return RSG_OK;
    if (ws_bytes < reduce_workspace_bytes(g, nst)) {
        set_error("reduction workspace too small: %zu < %zu", ws_bytes, reduce_workspace_bytes(g, nst));
        return RSG_ENOMEM;
    }
    if (nst > 65535) {
        set_error("reduction: at most 65535 orbitals per call");
        return RSG_EUNSUPPORTED;
    }
    const int64_t nblk = reduce_blocks(g.np);
    RArgs r;
    r.a = a;
    r.b = b;
    r.ijk = g.ijk;
    r.np = g.np;
    r.nst = nst;
    r.ldp = ldp;
    r.chunk = (g.np + nblk - 1) / nblk;
    r.h = g.h;
    r.axis = axis < 0 ? 0 : axis;
    r.off = 0.5 * (double)(g.n[r.axis] - 1);
    r.part = (double *)ws;
    const dim3 grid((unsigned)nblk, (unsigned)nst);
    if (kind == 0) k_reduce_partial<0><<<grid, RB, 0, s>>>(r);
    else if (kind == 1) k_reduce_partial<1><<<grid, RB, 0, s>>>(r);
    else if (kind == 3) k_reduce_partial<3><<<grid, RB, 0, s>>>(r);
    else k_reduce_partial<2><<<grid, RB, 0, s>>>(r);
    const double h3 = g.h * g.h * g.h;
    k_reduce_final<<<(unsigned)nst, RB, 0, s>>>(r.part, nblk, nst, (kind == 0 || kind == 3) ? 2 : 1, h3, out);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

int launch_pair_final(const double *P, int64_t nb, const double2 a[4], double h3, double *g, hipStream_t s) {
    k_pair_final<<<1, RB, 0, s>>>((const double2 *)P, nb, a[0], a[1], a[2], a[3], h3, g);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

int launch_mul_axis(const Grid &g, int axis, const double2 *src, double2 *dst, int64_t nst,
                    int64_t ldp, hipStream_t s) {
    if (nst == 0 || g.np == 0) return RSG_OK;
    if (nst > 65535) {
        set_error("pointwise: at most 65535 orbitals per call");
        return RSG_EUNSUPPORTED;
    }
    PwArgs a;
    a.src[0] = src;
    a.dst = dst;
    a.ijk = g.ijk;
    a.np = g.np;
    a.nst = nst;
    a.ldp = ldp;
    a.h = g.h;
    a.axis = axis;
    a.off = 0.5 * (double)(g.n[axis] - 1);
    k_mul_axis<<<pw_grid(g.np, nst), 256, 0, s>>>(a);
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

// ------------------------------------------------------------------------
// Allocation-free inner products: the partial sums live in a static device
// array instead of a caller workspace, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops).
// ------------------------------------------------------------------------

#include <mutex>

// 1 MiB: the partial sums of up to 64 orbitals at the largest partition
// (1024 workgroups per orbital), plus the per-orbital totals.  External
// linkage on purpose: a static device array gets a local symbol in the
// code object, which the runtime's symbol lookup does not find.
static constexpr size_t kScratchBytes = (size_t)1 << 20;
__device__ __align__(256) char rsg_noalloc_scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_addr;  // device ordinal -> address of that device's copy

// The device address of the scratch array on the current device, looked up once per
// device with that device current.  In host code the array's name is only a
// host-side stand-in; kernels get this address.
int scratch_address(void **out) {
    int dev = 0;
    RSG_CHECK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it == g_scratch_addr.end()) {
        void *p = nullptr;
        RSG_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(rsg_noalloc_scratch)));
        RSG_REQUIRE(p != nullptr, RSG_EHIP, "scratch: no device address");
        it = g_scratch_addr.emplace(dev, p).first;
    }
    *out = it->second;
    return RSG_OK;
}

}  // namespace

extern "C" size_t rsg_dot_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" int rsg_dot_noalloc(rsg_grid_t g, const void *a, const void *b, int64_t nst, int64_t ldp, double *out,
                               void *stream) {
    using namespace rsg;
    clear_error();
    RSG_REQUIRE(g, RSG_EINVAL, "rsg_dot_noalloc: null grid");
    RSG_REQUIRE(nst >= 0 && ldp >= 1 && ldp >= g->np, RSG_ESHAPE, "rsg_dot_noalloc: need nst >= 0 and ldp >= np");
    RSG_REQUIRE(nst == 0 || (a && b && out), RSG_EINVAL, "rsg_dot_noalloc: null pointer");
    RSG_REQUIRE((((uintptr_t)a | (uintptr_t)b) & 15) == 0, RSG_EINVAL, "rsg_dot_noalloc: pointer not 16-byte aligned");
    const size_t need = reduce_workspace_bytes(*g, nst);
    RSG_REQUIRE(need <= kScratchBytes, RSG_EUNSUPPORTED,
                "rsg_dot_noalloc: %lld orbitals on %lld slots need %zu scratch bytes, more than the %zu held",
                (long long)nst, (long long)g->np, need, kScratchBytes);
    if (nst == 0) return RSG_OK;
    void *ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    // every partial the final pass reads is written by the first pass of this
    // call, so nothing needs clearing
    return launch_reduce(*g, 0, 0, (const double2 *)a, (const double2 *)b, nst, ldp, out, ws, kScratchBytes,
                         (hipStream_t)stream);
}
