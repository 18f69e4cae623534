// C-ABI entry points: Hamiltonian handles, H*psi, Taylor(4) propagation,
// reductions, energy, the discrete adjoint and the checkpointed control
// gradient.  Everything numeric runs in the kernels of the other units; this
// file validates arguments, carves workspaces and orders launches.
#include "rsg_internal.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <set>
#include <tuple>

namespace rsg {

// Roots r_1..r_4 of the Taylor(4) polynomial T4(z) = sum_{k<=4} z^k / k!
// (of z^4 + 4 z^3 + 12 z^2 + 24 z + 24), largest modulus first: two
// conjugate pairs of moduli 2.52 and 1.94.  Durand-Kerner iteration from the
// usual spread start, then Newton steps on each root.
const std::complex<double> *taylor4_roots() {
    static std::complex<double> r[4];
    static std::once_flag once;
    std::call_once(once, [] {
        auto p = [](std::complex<double> z) { return (((z + 4.0) * z + 12.0) * z + 24.0) * z + 24.0; };
        auto dp = [](std::complex<double> z) { return ((4.0 * z + 12.0) * z + 24.0) * z + 24.0; };
        const std::complex<double> w(0.4, 0.9);
        for (int k = 0; k < 4; ++k) r[k] = std::pow(w, k);
        for (int it = 0; it < 500; ++it)
            for (int k = 0; k < 4; ++k) {
                std::complex<double> d = 1.0;
                for (int j = 0; j < 4; ++j)
                    if (j != k) d *= r[k] - r[j];
                r[k] -= p(r[k]) / d;
            }
        for (int k = 0; k < 4; ++k)
            for (int it = 0; it < 3; ++it) r[k] -= p(r[k]) / dp(r[k]);
        std::sort(r, r + 4, [](const std::complex<double> &a, const std::complex<double> &b) {
            return std::abs(a) != std::abs(b) ? std::abs(a) > std::abs(b) : a.imag() > b.imag();
        });
    });
    return r;
}

// Whether a step of this handle in dtype runs as the product of the four
// linear factors of T4 (FP64 without an absorber mask) or as 1 + z times
// the product of its cubic tail's factors (mixed precision, masked).
bool step_is_product(const Ham &H, int32_t dtype) { return dtype == RSG_C128 && !H.mask; }

// ------------------------------------------------------------------ errors

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

// ------------------------------------------------------------------ timing

namespace {
std::mutex g_tmu;
bool g_timing = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_events;
hipEvent_t g_pending = nullptr;

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}
}  // namespace

void timing_before(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing || capturing(s)) return;
    if (hipEventCreate(&g_pending) != hipSuccess) {
        g_pending = nullptr;
        return;
    }
    (void)hipEventRecord(g_pending, s);
}

void timing_after(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing || !g_pending) return;
    hipEvent_t e1;
    if (hipEventCreate(&e1) != hipSuccess) return;
    (void)hipEventRecord(e1, s);
    g_events.emplace_back(g_pending, e1);
    g_pending = nullptr;
}

// ------------------------------------------------------------ Ham lifetime

Ham::~Ham() {
    if (V) (void)hipFree(V);
    if (mask) (void)hipFree(mask);
    if (vim) (void)hipFree(vim);
    if (V32) (void)hipFree(V32);
    if (kb_idx) (void)hipFree(kb_idx);
    if (kb_p) (void)hipFree(kb_p);
    if (kb_p32) (void)hipFree(kb_p32);
    if (kb_E) (void)hipFree(kb_E);
    if (gather_items) (void)hipFree(gather_items);
    for (auto *p : scatter_items)
        if (p) (void)hipFree(p);
}

namespace {

__global__ void k_to_float(const double *src, float *dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

// Plain copy, four 16-byte loads in flight per thread per iteration.
__global__ void __launch_bounds__(256) k_copy16(const int4 *src, int4 *dst, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const int4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

__global__ void k_sum(const double *v, int64_t n, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += v[i];
    *out = s;
}

unsigned nblocks_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

}  // namespace

int check_batch(const Ham *H, const void *p, int64_t nst, int64_t ldp, const char *who) {
    RSG_REQUIRE(H, RSG_EINVAL, "%s: null Hamiltonian", who);
    RSG_REQUIRE(nst >= 0 && ldp >= 1 && ldp >= H->g->np, RSG_ESHAPE,
                "%s: need nst >= 0 and ldp >= np (ldp %lld, np %lld)", who, (long long)ldp,
                (long long)H->g->np);
    RSG_REQUIRE(p || nst == 0 || H->g->np == 0, RSG_EINVAL, "%s: null orbital pointer", who);
    RSG_REQUIRE(((uintptr_t)p & 15) == 0, RSG_EINVAL, "%s: orbital pointer not 16-byte aligned", who);
    return RSG_OK;
}

// --------------------------------------------------------- internal ops

// out = H(in), FP64.
int hpsi_impl(const Ham &H, const void *in, void *out, int64_t nst, int64_t ldp, double field,
              const double *field_dev, void *D, hipStream_t s) {
    int rc = launch_kb_gather(H, in, 0, 0, nst, ldp, D, s);
    if (rc) return rc;
    StageArgs a;
    a.in = in;
    a.out = out;
    a.mode = 0;
    a.nst = nst;
    a.ldp = ldp;
    a.field = field;
    a.field_dev = field_dev;
    rc = launch_stencil(H, a, H.tile_for(nst, 0), s);
    if (rc) return rc;
    return launch_kb_scatter(H, out, 0, 0, nst, ldp, D, 1.0, 0.0, nullptr, s);
}

namespace {

// One Taylor stage: out = base + c H(in) (base = in in a product-form step).
int stage_impl(const Ham &H, const void *in, int in_t, const void *base, void *out, int out_t,
               int compute, int64_t nst, int64_t ldp, double cre, double cim, double field,
               const double *field_dev, void *D, hipStream_t s, const double *mask = nullptr,
               const void *pair_y = nullptr, double *pair_out = nullptr) {
    int rc = launch_kb_gather(H, in, in_t, compute, nst, ldp, D, s);
    if (rc) return rc;
    StageArgs a;
    a.in = in;
    a.base = base;
    a.out = out;
    a.in_t = in_t;
    a.out_t = out_t;
    a.compute = compute;
    a.mode = 1;
    a.nst = nst;
    a.ldp = ldp;
    a.field = field;
    a.field_dev = field_dev;
    a.cre = cre;
    a.cim = cim;
    a.first = in == base;
    a.mask = mask;
    a.pair_y = pair_y;
    a.pair_out = pair_out;
    rc = launch_stencil(H, a, H.tile_for(nst, compute), s);
    if (rc) return rc;
    return launch_kb_scatter(H, out, out_t, compute, nst, ldp, D, cre, cim, mask, s);
}

size_t step_ws(const Ham &H, int64_t nst, int64_t ldp, int32_t dtype) {
    const size_t e = dtype == RSG_C128 ? 16 : 8;
    return 2 * rounded(batch_bytes(nst, ldp, e)) + rounded(kb_workspace_bytes(H, nst)) + 256;
}


// Coefficient a_k = i dt / r_k of the k-th linear factor 1 + a_k H of the
// Taylor(4) polynomial in -i dt H.
std::complex<double> factor_coef(int k, double dt) { return std::complex<double>(0.0, dt) / taylor4_roots()[k]; }

// Product-form step y[0] = F1 psi, y[1] = F2 y[0], y[2] = F3 y[1], psi_out =
// F4 y[2], F_k = 1 + a_k H; y[2] may alias y[0]; psi_out = NULL stops after
// the three stage outputs.  D: projector workspace.
int step_product(const Ham &H, const void *psi, void *const y[3], void *psi_out, int64_t nst, int64_t ldp,
                 double dt, double field, const double *field_dev, void *D, hipStream_t s) {
    const void *in[4] = {psi, y[0], y[1], y[2]};
    void *out[4] = {y[0], y[1], y[2], psi_out};
    for (int k = 0; k < (psi_out ? 4 : 3); ++k) {
        const std::complex<double> c = factor_coef(k, dt);
        const int rc = stage_impl(H, in[k], 0, in[k], out[k], 0, 0, nst, ldp, c.real(), c.imag(), field, field_dev,
                                  D, s);
        if (rc) return rc;
    }
    return RSG_OK;
}

// Roots s_1..s_3 of the cubic (T4(z) - 1) / z = 1 + z/2 + z^2/6 + z^3/24
// (of z^3 + 4 z^2 + 12 z + 24), the real root first; same method as the
// quartic's.
const std::complex<double> *taylor4_tail_roots() {
    static std::complex<double> r[3];
    static std::once_flag once;
    std::call_once(once, [] {
        auto p = [](std::complex<double> z) { return ((z + 4.0) * z + 12.0) * z + 24.0; };
        auto dp = [](std::complex<double> z) { return (3.0 * z + 8.0) * z + 12.0; };
        const std::complex<double> w(0.4, 0.9);
        for (int k = 0; k < 3; ++k) r[k] = std::pow(w, k);
        for (int it = 0; it < 500; ++it)
            for (int k = 0; k < 3; ++k) {
                std::complex<double> d = 1.0;
                for (int j = 0; j < 3; ++j)
                    if (j != k) d *= r[k] - r[j];
                r[k] -= p(r[k]) / d;
            }
        for (int k = 0; k < 3; ++k)
            for (int it = 0; it < 3; ++it) r[k] -= p(r[k]) / dp(r[k]);
        std::sort(r, r + 3, [](const std::complex<double> &a, const std::complex<double> &b) {
            return std::abs(a.imag()) != std::abs(b.imag()) ? std::abs(a.imag()) < std::abs(b.imag())
                                                            : a.imag() > b.imag();
        });
    });
    return r;
}

// Taylor(4) step psi_out <- T4(-i dt H) psi, z = -i dt H.
//  - FP64 without a mask: T4(z) = prod_k (1 - z / r_k) over its roots, so
//    the step is four stages y <- y + (i dt / r_k) H y.  Each stage reads
//    only its input (whose centre value is its own base term) and writes
//    one buffer: 32 B per point and orbital, against 48 for a stage that
//    also reads psi (Horner form).  The factor moduli stay below 2.2 up to the
//    stability limit dt |lambda| = 2 sqrt 2.
//  - Mixed precision and the masked step: T4(z) = 1 + z prod_j (1 - z/s_j)
//    over the roots of the cubic tail.  Three stages y <- y + (i dt / s_j)
//    H y from psi, then psi_out = psi + (-i dt) H y: psi enters only the
//    first and the last stage, so with complex64 work buffers psi itself
//    is carried in FP64 (the last stage adds the FP32 correction to it),
//    and the mask is applied by the last stage, which has psi as its base.
// Work buffers alternate; only the last stage writes psi_out, which may be
// psi itself (each output point reads only its own input value).
int step_impl(const Ham &H, const void *psi, void *psi_out, int64_t nst, int64_t ldp, int32_t dtype,
              double dt, double field, const double *field_dev, void *ws, size_t ws_bytes, hipStream_t s) {
    const size_t e = dtype == RSG_C128 ? 16 : 8;
    Carve c(ws, ws_bytes);
    void *w1 = c.take(batch_bytes(nst, ldp, e));
    void *w2 = c.take(batch_bytes(nst, ldp, e));
    void *D = c.take(kb_workspace_bytes(H, nst));
    if (!c.ok) {
        set_error("propagate: workspace too small (%zu < %zu bytes)", ws_bytes, step_ws(H, nst, ldp, dtype));
        return RSG_ENOMEM;
    }
    const int cmp = dtype == RSG_C128 ? 0 : 1;
    const int wt = dtype == RSG_C128 ? 0 : 1;  // work-buffer type
    int rc;
    if (step_is_product(H, dtype)) {
        void *y[3] = {w1, w2, w1};
        return step_product(H, psi, y, psi_out, nst, ldp, dt, field, field_dev, D, s);
    }
    const std::complex<double> *sr = taylor4_tail_roots();
    const void *in[3] = {psi, w1, w2};
    const int in_t[3] = {0, wt, wt};
    void *out[3] = {w1, w2, w1};
    for (int j = 0; j < 3; ++j) {
        const std::complex<double> cj = std::complex<double>(0.0, dt) / sr[j];  // i dt / s_j
        if ((rc = stage_impl(H, in[j], in_t[j], in[j], out[j], wt, cmp, nst, ldp, cj.real(), cj.imag(), field,
                             field_dev, D, s)))
            return rc;
    }
    // psi_out = M (psi + (-i dt) H y3), the mask if any
    return stage_impl(H, w1, wt, psi, psi_out, 0, cmp, nst, ldp, 0.0, -dt, field, field_dev, D, s, H.mask);
}

// Pair partials of one adjoint stage: one complex value per stencil
// workgroup of H's FP64 tile for nst orbitals.
int64_t adjoint_pair_blocks(const Ham &H, int64_t nst) {
    const int64_t nb = stencil_blocks(H, nst, 0, nullptr);
    return nb < 0 ? 0 : nb;
}

size_t adjoint_product_ws(const Ham &H, int64_t nst, int64_t ldp) {
    return 3 * rounded(batch_bytes(nst, ldp, 16)) + rounded(kb_workspace_bytes(H, nst)) +
           rounded(4 * (size_t)adjoint_pair_blocks(H, nst) * 16) + 256;
}

// Discrete adjoint of a product-form step psi_{n+1} = F4 F3 F2 F1 psi_n,
// F_k = 1 + a_k H(E_n), given y[0] = psi_n and the stage outputs y[1..3]
// (y[k] = F_k ... F_1 psi_n).  With m_4 = lambda_{n+1} and m_{k-1} =
// F_k^+ m_k (F_k^+ = 1 + conj(a_k) H, H Hermitian):
//   lambda_n = m_0,   dJ/dE_n = 2 Re sum_{k=1}^{4} a_k <m_k | x_axis | y[k-1]>,
// the derivative of the product by the rule for each factor (dF_k/dE =
// a_k x_axis).  Four first-type stencil stages on the costate; the stage
// that reads m_k also reads y[k-1] at each point and sums its pair term, so
// the pairs cost 16 B per point and orbital each and no separate pass; one
// small kernel adds the per-workgroup partials in a fixed order.
int adjoint_product_impl(const Ham &H, const void *const y[4], void *lambda, int64_t nst, int64_t ldp, double dt,
                         double field, const double *field_dev, double *g_dev, void *ws, size_t ws_bytes,
                         hipStream_t s) {
    Carve c(ws, ws_bytes);
    const size_t bb = batch_bytes(nst, ldp, 16);
    void *m[5];
    m[4] = lambda;
    for (int k = 1; k < 4; ++k) m[k] = c.take(bb);
    void *D = c.take(kb_workspace_bytes(H, nst));
    const int64_t nb = stencil_blocks(H, nst, 0, s);
    if (nb < 0) return (int)nb;
    double *P = (double *)c.take(4 * (size_t)nb * 16);
    if (!c.ok) {
        set_error("adjoint: workspace too small (%zu < %zu bytes)", ws_bytes, adjoint_product_ws(H, nst, ldp));
        return RSG_ENOMEM;
    }
    int rc;
    double2 ak[4];
    for (int k = 4; k >= 1; --k) {
        const std::complex<double> a = factor_coef(k - 1, dt);
        ak[k - 1] = make_double2(a.real(), a.imag());
        const std::complex<double> ca = std::conj(a);
        void *out = k > 1 ? m[k - 1] : lambda;  // lambda_{n+1} (= m_4) was read by the first of these stages
        if ((rc = stage_impl(H, m[k], 0, m[k], out, 0, 0, nst, ldp, ca.real(), ca.imag(), field, field_dev, D, s,
                             nullptr, y[k - 1], P + 2 * (size_t)nb * (k - 1))))
            return rc;
    }
    return launch_pair_final(P, nb, ak, H.g->h * H.g->h * H.g->h, g_dev, s);
}

// One adjoint step from psi_n alone: its three stage outputs recomputed
// into the workspace, then adjoint_product_impl.
size_t adjoint_ws(const Ham &H, int64_t nst, int64_t ldp) {
    return 3 * rounded(batch_bytes(nst, ldp, 16)) + adjoint_product_ws(H, nst, ldp) + 256;
}

int adjoint_step_impl(const Ham &H, const void *psi_n, void *lambda, int64_t nst, int64_t ldp, double dt,
                      double field, double *g_dev, void *ws, size_t ws_bytes, hipStream_t s) {
    Carve c(ws, ws_bytes);
    const size_t bb = batch_bytes(nst, ldp, 16);
    void *y[3] = {c.take(bb), c.take(bb), c.take(bb)};
    size_t rest = 0;
    void *aws = c.take_rest(&rest);
    if (!c.ok) {
        set_error("adjoint: workspace too small (%zu < %zu bytes)", ws_bytes, adjoint_ws(H, nst, ldp));
        return RSG_ENOMEM;
    }
    int rc = step_product(H, psi_n, y, nullptr, nst, ldp, dt, field, nullptr, aws, s);
    if (rc) return rc;
    const void *yy[4] = {psi_n, y[0], y[1], y[2]};
    return adjoint_product_impl(H, yy, lambda, nst, ldp, dt, field, nullptr, g_dev, aws, rest, s);
}

// Graph cache key for rsg_propagate.
struct GraphKey {
    const void *psi;
    int64_t nst, ldp;
    int32_t dtype;
    double dt;
    int64_t nsteps;
    const double *fields;
    const void *ws;
    size_t ws_bytes;
    hipStream_t stream;
    bool operator<(const GraphKey &o) const {
        return std::tie(psi, nst, ldp, dtype, dt, nsteps, fields, ws, ws_bytes, stream) <
               std::tie(o.psi, o.nst, o.ldp, o.dtype, o.dt, o.nsteps, o.fields, o.ws, o.ws_bytes,
                        o.stream);
    }
};

std::mutex g_graph_mu;
std::map<const Ham *, std::map<GraphKey, hipGraphExec_t>> g_graphs;

void drop_graphs(const Ham *H) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(H);
    if (it == g_graphs.end()) return;
    for (auto &kv : it->second) (void)hipGraphExecDestroy(kv.second);
    g_graphs.erase(it);
}

}  // namespace

}  // namespace rsg

using namespace rsg;

// ------------------------------------------------------------------- ABI

extern "C" const char *rsg_last_error(void) { return g_err; }
extern "C" const char *rsg_version(void) { return "rsg 0.1 (gfx950)"; }

extern "C" int rsg_ham_create(rsg_grid_t g, const double *vloc_dev, double kin, int32_t axis,
                              int32_t natoms, const rsg_proj_desc *proj, rsg_ham_t *out) {
    clear_error();
    RSG_REQUIRE(g && out, RSG_EINVAL, "rsg_ham_create: null argument");
    RSG_REQUIRE(axis >= -1 && axis <= 2, RSG_EINVAL, "rsg_ham_create: dipole_axis must be -1..2");
    RSG_REQUIRE(natoms >= 0 && (natoms == 0 || proj), RSG_EINVAL, "rsg_ham_create: bad projector list");
    RSG_REQUIRE(std::isfinite(kin), RSG_EINVAL, "rsg_ham_create: kinetic prefactor not finite");
    for (int a = 0; a < natoms; ++a) {
        RSG_REQUIRE(proj[a].n_support >= 0, RSG_EINVAL, "rsg_ham_create: atom %d negative support", a);
        RSG_REQUIRE(proj[a].n_support == 0 || (proj[a].idx && proj[a].p), RSG_EINVAL,
                    "rsg_ham_create: atom %d null projector table", a);
        RSG_REQUIRE(proj[a].n_support <= g->np, RSG_EINVAL, "rsg_ham_create: atom %d support larger than grid", a);
    }
    return guarded([&]() -> int {
        auto *H = new rsg_ham_s();
        H->g = g;
        H->kin = kin;
        H->axis = axis;
        H->natoms = natoms;
        auto fail = [&](const char *what, hipError_t e) {
            set_error("rsg_ham_create: %s: %s", what, hipGetErrorString(e));
            delete H;
            return RSG_EHIP;
        };
        hipError_t e;
        const int64_t np = g->np;
        // the kernels always read V (zeros when none is given)
        {
            const int64_t nv = np > 0 ? np : 1;
            if ((e = hipMalloc(&H->V, sizeof(double) * nv)) != hipSuccess) return fail("V", e);
            if ((e = hipMalloc(&H->V32, sizeof(float) * nv)) != hipSuccess) return fail("V32", e);
            if (vloc_dev && np > 0) {
                if ((e = hipMemcpy(H->V, vloc_dev, sizeof(double) * np, hipMemcpyDeviceToDevice)) != hipSuccess)
                    return fail("V copy", e);
            } else if ((e = hipMemset(H->V, 0, sizeof(double) * nv)) != hipSuccess) {
                return fail("V clear", e);
            }
            k_to_float<<<nblocks_for(nv), 256>>>(H->V, H->V32, nv);
        }
        if (natoms > 0) {
            // pad every support to a multiple of 16 entries (p = 0, index of
            // the atom's first point, or 0 for an empty support)
            H->kb_off.assign(natoms + 1, 0);
            H->kb_len.assign(natoms, 0);
            for (int a = 0; a < natoms; ++a) {
                H->kb_len[a] = proj[a].n_support;
                const int64_t padded = std::max<int64_t>(16, (proj[a].n_support + 15) / 16 * 16);
                H->kb_off[a + 1] = H->kb_off[a] + padded;
            }
            const int64_t total = H->kb_off[natoms];
            std::vector<int32_t> idx_h(total, 0);
            std::vector<double> p_h((size_t)total * 4, 0.0);
            std::vector<double> E_h((size_t)natoms * 4);
            for (int a = 0; a < natoms; ++a) {
                const int64_t n = proj[a].n_support;
                if (n > 0) {
                    if ((e = hipMemcpy(idx_h.data() + H->kb_off[a], proj[a].idx, sizeof(int32_t) * n,
                                       hipMemcpyDeviceToHost)) != hipSuccess)
                        return fail("projector index copy", e);
                    if ((e = hipMemcpy(p_h.data() + 4 * H->kb_off[a], proj[a].p, sizeof(double) * 4 * n,
                                       hipMemcpyDeviceToHost)) != hipSuccess)
                        return fail("projector value copy", e);
                }
                for (int64_t k = n; k < H->kb_off[a + 1] - H->kb_off[a]; ++k)
                    idx_h[H->kb_off[a] + k] = n > 0 ? idx_h[H->kb_off[a]] : 0;
                for (int i = 0; i < 4; ++i) E_h[4 * a + i] = proj[a].E[i];
            }
            // validate indices: in range and distinct within an atom
            std::vector<int32_t> mark(np > 0 ? np : 1, -1);
            for (int a = 0; a < natoms; ++a)
                for (int64_t k = 0; k < H->kb_len[a]; ++k) {
                    const int32_t r = idx_h[H->kb_off[a] + k];
                    if (r < 0 || r >= np) {
                        set_error("rsg_ham_create: atom %d projector index %d outside [0, %lld)", a, r,
                                  (long long)np);
                        delete H;
                        return RSG_EINVAL;
                    }
                    if (mark[r] == a) {
                        set_error("rsg_ham_create: atom %d lists point %d twice", a, r);
                        delete H;
                        return RSG_EINVAL;
                    }
                    mark[r] = a;
                }
            // greedy colouring: atoms whose supports overlap get different
            // colours, so one scatter launch never updates a point twice
            std::vector<int> colour(natoms, -1);
            std::vector<std::vector<char>> used;
            for (int a = 0; a < natoms; ++a) {
                int c = 0;
                for (;; ++c) {
                    if (c == (int)used.size()) used.emplace_back(np > 0 ? np : 1, 0);
                    bool clash = false;
                    for (int64_t k = 0; k < H->kb_len[a] && !clash; ++k)
                        clash = used[c][idx_h[H->kb_off[a] + k]] != 0;
                    if (!clash) break;
                }
                colour[a] = c;
                for (int64_t k = 0; k < H->kb_len[a]; ++k) used[c][idx_h[H->kb_off[a] + k]] = 1;
            }
            std::vector<int4> atoms(natoms);
            std::vector<std::vector<int2>> sc(used.size());
            for (int a = 0; a < natoms; ++a) {
                const int64_t padded = H->kb_off[a + 1] - H->kb_off[a];
                atoms[a] = make_int4((int)H->kb_off[a], (int)padded, (int)H->kb_len[a], a);
                for (int64_t k = 0; k < H->kb_len[a]; k += 16)
                    sc[colour[a]].push_back(make_int2(a, (int)(H->kb_off[a] + k)));
            }
            if ((e = hipMalloc(&H->kb_idx, sizeof(int32_t) * total)) != hipSuccess) return fail("idx", e);
            if ((e = hipMalloc(&H->kb_p, sizeof(double) * 4 * total)) != hipSuccess) return fail("p", e);
            if ((e = hipMalloc(&H->kb_p32, sizeof(float) * 4 * total)) != hipSuccess) return fail("p32", e);
            if ((e = hipMalloc(&H->kb_E, sizeof(double) * 4 * natoms)) != hipSuccess) return fail("E", e);
            if ((e = hipMalloc(&H->gather_items, sizeof(int4) * natoms)) != hipSuccess) return fail("atoms", e);
            if ((e = hipMemcpy(H->kb_idx, idx_h.data(), sizeof(int32_t) * total, hipMemcpyHostToDevice)) != hipSuccess)
                return fail("idx upload", e);
            if ((e = hipMemcpy(H->kb_p, p_h.data(), sizeof(double) * 4 * total, hipMemcpyHostToDevice)) != hipSuccess)
                return fail("p upload", e);
            if ((e = hipMemcpy(H->kb_E, E_h.data(), sizeof(double) * 4 * natoms, hipMemcpyHostToDevice)) != hipSuccess)
                return fail("E upload", e);
            if ((e = hipMemcpy(H->gather_items, atoms.data(), sizeof(int4) * natoms, hipMemcpyHostToDevice)) != hipSuccess)
                return fail("atom upload", e);
            k_to_float<<<nblocks_for(4 * total), 256>>>(H->kb_p, H->kb_p32, 4 * total);
            for (auto &v : sc) {
                int2 *d = nullptr;
                if (!v.empty()) {
                    if ((e = hipMalloc(&d, sizeof(int2) * v.size())) != hipSuccess) return fail("scatter", e);
                    if ((e = hipMemcpy(d, v.data(), sizeof(int2) * v.size(), hipMemcpyHostToDevice)) != hipSuccess) {
                        (void)hipFree(d);
                        return fail("scatter upload", e);
                    }
                }
                H->scatter_items.push_back(d);
                H->scatter_counts.push_back((int32_t)v.size());
            }
        }
        if ((e = hipGetLastError()) != hipSuccess) return fail("conversion", e);
        if ((e = hipDeviceSynchronize()) != hipSuccess) return fail("sync", e);
        *out = H;
        return RSG_OK;
    });
}

extern "C" int rsg_ham_destroy(rsg_ham_t H) {
    clear_error();
    if (H) drop_graphs(H);
    delete H;
    return RSG_OK;
}

extern "C" int rsg_ham_set_complex_scaling(rsg_ham_t H, double theta, const double *vim_dev) {
    clear_error();
    RSG_REQUIRE(H, RSG_EINVAL, "rsg_ham_set_complex_scaling: null Hamiltonian");
    RSG_REQUIRE(std::isfinite(theta), RSG_EINVAL, "rsg_ham_set_complex_scaling: theta not finite");
    const bool on = theta != 0 || vim_dev;
    RSG_REQUIRE(!on || H->natoms == 0, RSG_EUNSUPPORTED,
                "rsg_ham_set_complex_scaling: projectors are not complex-scaled in this library");
    RSG_REQUIRE(!on || !H->mask, RSG_EUNSUPPORTED,
                "rsg_ham_set_complex_scaling: a complex-scaled Hamiltonian takes no absorber mask");
    drop_graphs(H);  // captured steps hold the old kernels
    H->cs_theta = theta;
    if (!vim_dev) {
        if (H->vim) RSG_CHECK_HIP(hipFree(H->vim));
        H->vim = nullptr;
        return RSG_OK;
    }
    const int64_t np = H->g->np;
    if (!H->vim && np > 0) RSG_CHECK_HIP(hipMalloc(&H->vim, sizeof(double) * np));
    if (np > 0) RSG_CHECK_HIP(hipMemcpy(H->vim, vim_dev, sizeof(double) * np, hipMemcpyDeviceToDevice));
    return RSG_OK;
}

extern "C" int rsg_ham_set_mask(rsg_ham_t H, const double *mask_dev) {
    clear_error();
    RSG_REQUIRE(H, RSG_EINVAL, "rsg_ham_set_mask: null Hamiltonian");
    RSG_REQUIRE(!mask_dev || !H->complex_scaled(), RSG_EUNSUPPORTED,
                "rsg_ham_set_mask: a complex-scaled Hamiltonian takes no absorber mask");
    drop_graphs(H);  // captured steps hold the old mask (or none)
    if (!mask_dev) {
        if (H->mask) RSG_CHECK_HIP(hipFree(H->mask));
        H->mask = nullptr;
        return RSG_OK;
    }
    const int64_t np = H->g->np;
    if (!H->mask && np > 0) RSG_CHECK_HIP(hipMalloc(&H->mask, sizeof(double) * np));
    if (np > 0) {
        RSG_CHECK_HIP(hipMemcpy(H->mask, mask_dev, sizeof(double) * np, hipMemcpyDeviceToDevice));
    }
    return RSG_OK;
}

extern "C" size_t rsg_workspace_bytes(rsg_ham_t H, int32_t op, int64_t nst, int64_t ldp, int32_t dtype) {
    if (!H || nst < 0 || ldp < 1) return 0;
    switch (op) {
        case RSG_OP_HPSI: return rounded(kb_workspace_bytes(*H, nst)) + 256;
        case RSG_OP_STEP: return step_ws(*H, nst, ldp, dtype);
        case RSG_OP_REDUCE: return reduce_workspace_bytes(*H->g, nst);
        case RSG_OP_ENERGY:
            return rounded(batch_bytes(nst, ldp, 16)) + rounded(kb_workspace_bytes(*H, nst)) +
                   rounded(reduce_workspace_bytes(*H->g, nst)) + 256;
        case RSG_OP_ADJOINT: return adjoint_ws(*H, nst, ldp);
        default: return 0;
    }
}

extern "C" int rsg_hpsi(rsg_ham_t H, const void *psi, void *hpsi, int64_t nst, int64_t ldp,
                        int32_t dtype, double field, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = check_batch(H, psi, nst, ldp, "rsg_hpsi");
    if (rc) return rc;
    RSG_REQUIRE(dtype == RSG_C128, dtype == RSG_C64_MIXED ? RSG_EUNSUPPORTED : RSG_EDTYPE,
                "rsg_hpsi: dtype must be RSG_C128");
    RSG_REQUIRE(hpsi || nst == 0, RSG_EINVAL, "rsg_hpsi: null output");
    RSG_REQUIRE(((uintptr_t)hpsi & 15) == 0, RSG_EINVAL, "rsg_hpsi: output not 16-byte aligned");
    const size_t bb = batch_bytes(nst, ldp, 16);
    const char *a0 = (const char *)psi, *b0 = (const char *)hpsi;
    RSG_REQUIRE(nst == 0 || a0 + bb <= b0 || b0 + bb <= a0, RSG_EINVAL, "rsg_hpsi: psi and hpsi overlap");
    Carve c(ws, ws_bytes);
    void *D = c.take(kb_workspace_bytes(*H, nst));
    RSG_REQUIRE(c.ok, RSG_ENOMEM, "rsg_hpsi: workspace too small");
    if (nst == 0 || H->g->np == 0) return RSG_OK;
    return hpsi_impl(*H, psi, hpsi, nst, ldp, field, nullptr, D, (hipStream_t)stream);
}

extern "C" int rsg_propagate_step(rsg_ham_t H, void *psi, int64_t nst, int64_t ldp, int32_t dtype,
                                  double dt, double field, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = check_batch(H, psi, nst, ldp, "rsg_propagate_step");
    if (rc) return rc;
    RSG_REQUIRE(dtype == RSG_C128 || dtype == RSG_C64_MIXED, RSG_EDTYPE, "rsg_propagate_step: bad dtype %d", dtype);
    RSG_REQUIRE(dtype == RSG_C128 || !H->complex_scaled(), RSG_EUNSUPPORTED,
                "rsg_propagate_step: a complex-scaled Hamiltonian needs RSG_C128");
    RSG_REQUIRE(std::isfinite(dt) && std::isfinite(field), RSG_EINVAL, "rsg_propagate_step: dt/field not finite");
    RSG_REQUIRE(ws_bytes >= step_ws(*H, nst, ldp, dtype) - 256 || nst == 0, RSG_ENOMEM,
                "rsg_propagate_step: workspace too small (%zu < %zu)", ws_bytes, step_ws(*H, nst, ldp, dtype));
    if (nst == 0 || H->g->np == 0) return RSG_OK;
    return step_impl(*H, psi, psi, nst, ldp, dtype, dt, field, nullptr, ws, ws_bytes, (hipStream_t)stream);
}

extern "C" int rsg_propagate(rsg_ham_t H, void *psi, int64_t nst, int64_t ldp, int32_t dtype, double dt,
                             int64_t nsteps, const double *fields_dev, int32_t use_graph, void *ws,
                             size_t ws_bytes, void *stream) {
    clear_error();
    int rc = check_batch(H, psi, nst, ldp, "rsg_propagate");
    if (rc) return rc;
    RSG_REQUIRE(dtype == RSG_C128 || dtype == RSG_C64_MIXED, RSG_EDTYPE, "rsg_propagate: bad dtype %d", dtype);
    RSG_REQUIRE(dtype == RSG_C128 || !H->complex_scaled(), RSG_EUNSUPPORTED,
                "rsg_propagate: a complex-scaled Hamiltonian needs RSG_C128");
    RSG_REQUIRE(nsteps >= 0 && std::isfinite(dt), RSG_EINVAL, "rsg_propagate: bad nsteps/dt");
    RSG_REQUIRE(ws_bytes >= step_ws(*H, nst, ldp, dtype) - 256 || nst == 0, RSG_ENOMEM,
                "rsg_propagate: workspace too small (%zu < %zu)", ws_bytes, step_ws(*H, nst, ldp, dtype));
    if (nst == 0 || H->g->np == 0 || nsteps == 0) return RSG_OK;
    hipStream_t s = (hipStream_t)stream;
    auto run = [&]() -> int {
        for (int64_t n = 0; n < nsteps; ++n) {
            const int r = step_impl(*H, psi, psi, nst, ldp, dtype, dt, 0.0, fields_dev ? fields_dev + n : nullptr,
                                    ws, ws_bytes, s);
            if (r) return r;
        }
        return RSG_OK;
    };
    if (!use_graph) return run();
    RSG_REQUIRE(s != nullptr, RSG_EINVAL, "rsg_propagate: graph capture needs a non-default stream");
    // make sure every launch plan exists before capture (plan creation syncs)
    int err = RSG_OK;
    for (int cmp = 0; cmp < 2; ++cmp)
        if (!H->g->plan(launch_shape(*H, H->tile_for(nst, cmp)), s, &err)) return err;
    GraphKey key{psi, nst, ldp, dtype, dt, nsteps, fields_dev, ws, ws_bytes, s};
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        auto &m = g_graphs[H];
        auto it = m.find(key);
        if (it != m.end()) exec = it->second;
    }
    if (!exec) {
        RSG_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const int r = run();
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &graph);
        if (r) {
            if (graph) (void)hipGraphDestroy(graph);
            return r;
        }
        if (e != hipSuccess) {
            set_error("rsg_propagate: capture failed: %s", hipGetErrorString(e));
            return RSG_EHIP;
        }
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            set_error("rsg_propagate: graph instantiate failed: %s", hipGetErrorString(ei));
            return RSG_EHIP;
        }
        std::lock_guard<std::mutex> lk(g_graph_mu);
        g_graphs[H][key] = exec;
    }
    RSG_CHECK_HIP(hipGraphLaunch(exec, s));
    return RSG_OK;
}

static int check_reduce(const Grid *g, const void *a, int64_t nst, int64_t ldp, const void *out, const char *who) {
    RSG_REQUIRE(g, RSG_EINVAL, "%s: null grid", who);
    RSG_REQUIRE(nst >= 0 && ldp >= 1 && ldp >= g->np, RSG_ESHAPE, "%s: need nst >= 0 and ldp >= np", who);
    RSG_REQUIRE(nst == 0 || (a && out), RSG_EINVAL, "%s: null pointer", who);
    RSG_REQUIRE(((uintptr_t)a & 15) == 0, RSG_EINVAL, "%s: pointer not 16-byte aligned", who);
    return RSG_OK;
}

extern "C" size_t rsg_reduce_workspace_bytes(rsg_grid_t g, int64_t nst) {
    if (!g || nst < 0) return 0;
    return reduce_workspace_bytes(*g, nst);
}

extern "C" int rsg_dot(rsg_grid_t g, const void *a, const void *b, int64_t nst, int64_t ldp, double *out,
                       void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = check_reduce(g, a, nst, ldp, out, "rsg_dot");
    if (rc) return rc;
    RSG_REQUIRE(nst == 0 || b, RSG_EINVAL, "rsg_dot: null pointer");
    RSG_REQUIRE(((uintptr_t)b & 15) == 0, RSG_EINVAL, "rsg_dot: pointer not 16-byte aligned");
    return launch_reduce(*g, 0, 0, (const double2 *)a, (const double2 *)b, nst, ldp, out, ws, ws_bytes,
                         (hipStream_t)stream);
}

extern "C" int rsg_bilinear(rsg_grid_t g, const void *a, const void *b, int64_t nst, int64_t ldp, double *out,
                            void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = check_reduce(g, a, nst, ldp, out, "rsg_bilinear");
    if (rc) return rc;
    RSG_REQUIRE(nst == 0 || b, RSG_EINVAL, "rsg_bilinear: null pointer");
    RSG_REQUIRE(((uintptr_t)b & 15) == 0, RSG_EINVAL, "rsg_bilinear: pointer not 16-byte aligned");
    return launch_reduce(*g, 3, 0, (const double2 *)a, (const double2 *)b, nst, ldp, out, ws, ws_bytes,
                         (hipStream_t)stream);
}

extern "C" int rsg_norm2(rsg_grid_t g, const void *a, int64_t nst, int64_t ldp, double *out, void *ws,
                         size_t ws_bytes, void *stream) {
    clear_error();
    int rc = check_reduce(g, a, nst, ldp, out, "rsg_norm2");
    if (rc) return rc;
    return launch_reduce(*g, 1, 0, (const double2 *)a, nullptr, nst, ldp, out, ws, ws_bytes,
                         (hipStream_t)stream);
}

extern "C" int rsg_dipole_expectation(rsg_ham_t H, const void *a, int64_t nst, int64_t ldp, double *out,
                                      void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    RSG_REQUIRE(H, RSG_EINVAL, "rsg_dipole_expectation: null Hamiltonian");
    RSG_REQUIRE(H->axis >= 0, RSG_EINVAL, "rsg_dipole_expectation: Hamiltonian has no dipole axis");
    int rc = check_reduce(H->g, a, nst, ldp, out, "rsg_dipole_expectation");
    if (rc) return rc;
    return launch_reduce(*H->g, 2, H->axis, (const double2 *)a, nullptr, nst, ldp, out, ws, ws_bytes,
                         (hipStream_t)stream);
}

extern "C" int rsg_energy(rsg_ham_t H, const void *psi, int64_t nst, int64_t ldp, int32_t dtype, double field,
                          double *out, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = check_batch(H, psi, nst, ldp, "rsg_energy");
    if (rc) return rc;
    RSG_REQUIRE(dtype == RSG_C128, RSG_EDTYPE, "rsg_energy: dtype must be RSG_C128");
    RSG_REQUIRE(nst == 0 || out, RSG_EINVAL, "rsg_energy: null output");
    Carve c(ws, ws_bytes);
    void *hp = c.take(batch_bytes(nst, ldp, 16));
    void *D = c.take(kb_workspace_bytes(*H, nst));
    const size_t rb = reduce_workspace_bytes(*H->g, nst);
    void *R = c.take(rb);
    RSG_REQUIRE(c.ok, RSG_ENOMEM, "rsg_energy: workspace too small");
    if (nst == 0) return RSG_OK;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = hpsi_impl(*H, psi, hp, nst, ldp, field, nullptr, D, s))) return rc;
    return launch_reduce(*H->g, 0, 0, (const double2 *)psi, (const double2 *)hp, nst, ldp, out, R, rb, s);
}

extern "C" int rsg_adjoint_step(rsg_ham_t H, const void *psi_n, void *lambda, int64_t nst, int64_t ldp,
                                double dt, double field, double *g_dev, void *ws, size_t ws_bytes,
                                void *stream) {
    clear_error();
    int rc = check_batch(H, psi_n, nst, ldp, "rsg_adjoint_step");
    if (rc) return rc;
    rc = check_batch(H, lambda, nst, ldp, "rsg_adjoint_step");
    if (rc) return rc;
    RSG_REQUIRE(H->axis >= 0, RSG_EINVAL, "rsg_adjoint_step: Hamiltonian has no dipole axis");
    RSG_REQUIRE(!H->mask, RSG_EUNSUPPORTED, "rsg_adjoint_step: the adjoint of a masked step is not built");
    RSG_REQUIRE(!H->complex_scaled(), RSG_EUNSUPPORTED,
                "rsg_adjoint_step: the adjoint assumes a Hermitian Hamiltonian (no complex scaling)");
    RSG_REQUIRE(g_dev, RSG_EINVAL, "rsg_adjoint_step: null gradient output");
    RSG_REQUIRE(ws_bytes >= adjoint_ws(*H, nst, ldp) - 256, RSG_ENOMEM,
                "rsg_adjoint_step: workspace too small (%zu < %zu)", ws_bytes, adjoint_ws(*H, nst, ldp));
    RSG_REQUIRE(nst > 0, RSG_ESHAPE, "rsg_adjoint_step: nst must be > 0");
    return adjoint_step_impl(*H, psi_n, lambda, nst, ldp, dt, field, g_dev, ws, ws_bytes, (hipStream_t)stream);
}

// The control entry points take handles without mask or complex scaling,
// whose steps run in product form.  Full workspace: the segment store keeps,
// per step, the state and its three stage outputs (the adjoint reads them).
// Minimum workspace: the states only, plus three batches into which each
// adjoint step recomputes its stage outputs.  Both need three batches for
// the adjoint itself.
static size_t control_ws_head(int64_t nst, int64_t ldp, int64_t nsteps) {
    return rounded(sizeof(double) * (size_t)std::max<int64_t>(nsteps, 1)) * 2 + rounded(sizeof(double) * (size_t)nst) +
           rounded(batch_bytes(nst, ldp, 16));
}
static size_t control_ws_tail(const Ham &H, int64_t nst, int64_t ldp) {
    return std::max({step_ws(H, nst, ldp, RSG_C128), rounded(kb_workspace_bytes(H, nst)) + 256,
                     adjoint_product_ws(H, nst, ldp)}) +
           256;
}
static size_t control_ws(const Ham &H, int64_t nst, int64_t ldp, int64_t nsteps, int64_t ckpt) {
    const size_t bb = rounded(batch_bytes(nst, ldp, 16));
    return control_ws_head(nst, ldp, nsteps) + 4 * (size_t)std::max<int64_t>(ckpt, 1) * bb +
           control_ws_tail(H, nst, ldp);
}
static size_t control_ws_min(const Ham &H, int64_t nst, int64_t ldp, int64_t nsteps, int64_t ckpt) {
    const size_t bb = rounded(batch_bytes(nst, ldp, 16));
    return control_ws_head(nst, ldp, nsteps) + ((size_t)std::max<int64_t>(ckpt, 1) + 3) * bb +
           control_ws_tail(H, nst, ldp);
}

extern "C" size_t rsg_control_workspace_bytes(rsg_ham_t H, int64_t nst, int64_t ldp, int64_t nsteps,
                                              int64_t ckpt_every) {
    if (!H || nst < 0 || ldp < 1 || nsteps < 0 || ckpt_every < 1) return 0;
    return control_ws(*H, nst, ldp, nsteps, ckpt_every);
}

extern "C" size_t rsg_control_workspace_bytes_min(rsg_ham_t H, int64_t nst, int64_t ldp, int64_t nsteps,
                                                  int64_t ckpt_every) {
    if (!H || nst < 0 || ldp < 1 || nsteps < 0 || ckpt_every < 1) return 0;
    return control_ws_min(*H, nst, ldp, nsteps, ckpt_every);
}

static int check_control(rsg_ham_t H, const void *psi, int64_t nst, int64_t ldp, double dt, int64_t nsteps,
                         const double *coef, int32_t ncoef, int64_t ckpt, size_t ws_bytes, const char *who) {
    int rc = check_batch(H, psi, nst, ldp, who);
    if (rc) return rc;
    RSG_REQUIRE(H->axis >= 0, RSG_EINVAL, "%s: Hamiltonian has no dipole axis", who);
    RSG_REQUIRE(!H->mask, RSG_EUNSUPPORTED, "%s: the adjoint of a masked step is not built", who);
    RSG_REQUIRE(!H->complex_scaled(), RSG_EUNSUPPORTED,
                "%s: the adjoint assumes a Hermitian Hamiltonian (no complex scaling)", who);
    RSG_REQUIRE(nst > 0 && nsteps > 0 && dt > 0 && std::isfinite(dt), RSG_EINVAL, "%s: need nst, nsteps, dt > 0", who);
    RSG_REQUIRE(ncoef >= 0 && (ncoef == 0 || coef), RSG_EINVAL, "%s: bad coefficient array", who);
    RSG_REQUIRE(ckpt >= 1, RSG_EINVAL, "%s: ckpt_every must be >= 1", who);
    RSG_REQUIRE(ws_bytes >= control_ws_min(*H, nst, ldp, nsteps, ckpt) - 256, RSG_ENOMEM,
                "%s: workspace too small (%zu < %zu)", who, ws_bytes, control_ws_min(*H, nst, ldp, nsteps, ckpt));
    return RSG_OK;
}

extern "C" int rsg_control_forward(rsg_ham_t H, void *psi, int64_t nst, int64_t ldp, double dt, int64_t nsteps,
                                   const double *coef, int32_t ncoef, int64_t ckpt_every, void *ckpt_dev,
                                   double *J_dev, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = check_control(H, psi, nst, ldp, dt, nsteps, coef, ncoef, ckpt_every, ws_bytes, "rsg_control_forward");
    if (rc) return rc;
    RSG_REQUIRE(J_dev, RSG_EINVAL, "rsg_control_forward: null J output");
    hipStream_t s = (hipStream_t)stream;
    const double T = dt * (double)nsteps;
    const size_t bb = batch_bytes(nst, ldp, 16);
    Carve c(ws, ws_bytes);
    double *fields = (double *)c.take(sizeof(double) * nsteps);
    (void)c.take(sizeof(double) * nsteps);
    double *per = (double *)c.take(sizeof(double) * nst);
    (void)c.take(bb);
    (void)c.take(std::max<int64_t>(ckpt_every, 1) * rounded(bb));
    size_t rest = 0;
    void *sws = c.take_rest(&rest);
    if (!c.ok) {
        set_error("rsg_control_forward: workspace carve failed");
        return RSG_ENOMEM;
    }
    if ((rc = rsg_laser_field(coef, ncoef, T, dt, 0, nsteps, fields, stream))) return rc;
    if (ckpt_dev) RSG_CHECK_HIP(hipMemcpyAsync(ckpt_dev, psi, bb, hipMemcpyDeviceToDevice, s));
    for (int64_t n = 0; n < nsteps; ++n) {
        if ((rc = step_impl(*H, psi, psi, nst, ldp, RSG_C128, dt, 0.0, fields + n, sws, rest, s))) return rc;
        if (ckpt_dev && (n + 1) % ckpt_every == 0)
            RSG_CHECK_HIP(hipMemcpyAsync((char *)ckpt_dev + (size_t)((n + 1) / ckpt_every) * bb, psi, bb,
                                         hipMemcpyDeviceToDevice, s));
    }
    const size_t rb = reduce_workspace_bytes(*H->g, nst);
    if ((rc = launch_reduce(*H->g, 2, H->axis, (const double2 *)psi, nullptr, nst, ldp, per, sws, rb, s))) return rc;
    k_sum<<<1, 64, 0, s>>>(per, nst, J_dev);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

extern "C" int rsg_control_backward(rsg_ham_t H, const void *psi_T, int64_t nst, int64_t ldp, double dt,
                                    int64_t nsteps, const double *coef, int32_t ncoef, int64_t ckpt_every,
                                    const void *ckpt_dev, double *grad_dev, double *g_steps_dev, void *ws,
                                    size_t ws_bytes, void *stream) {
    clear_error();
    int rc = check_control(H, psi_T, nst, ldp, dt, nsteps, coef, ncoef, ckpt_every, ws_bytes, "rsg_control_backward");
    if (rc) return rc;
    RSG_REQUIRE(ckpt_dev, RSG_EINVAL, "rsg_control_backward: null checkpoint store");
    RSG_REQUIRE(ncoef == 0 || grad_dev, RSG_EINVAL, "rsg_control_backward: null gradient output");
    hipStream_t s = (hipStream_t)stream;
    const double T = dt * (double)nsteps;
    const size_t bb = batch_bytes(nst, ldp, 16);
    const size_t bbr = rounded(bb);
    Carve c(ws, ws_bytes);
    double *fields = (double *)c.take(sizeof(double) * nsteps);
    double *gs = (double *)c.take(sizeof(double) * nsteps);
    (void)c.take(sizeof(double) * nst);
    void *lam = c.take(bb);
    char *states = (char *)c.take(std::max<int64_t>(ckpt_every, 1) * bbr);
    // the full workspace keeps every step's stage outputs; the minimum one
    // has room for one step's, recomputed by each adjoint step
    const bool keep = ws_bytes + 256 >= control_ws(*H, nst, ldp, nsteps, ckpt_every);
    char *ystore = (char *)c.take((keep ? 3 * std::max<int64_t>(ckpt_every, 1) : 3) * bbr);
    size_t rest = 0;
    void *sws = c.take_rest(&rest);
    if (!c.ok) {
        set_error("rsg_control_backward: workspace carve failed");
        return RSG_ENOMEM;
    }
    if (g_steps_dev) gs = g_steps_dev;
    if ((rc = rsg_laser_field(coef, ncoef, T, dt, 0, nsteps, fields, stream))) return rc;
    if ((rc = launch_mul_axis(*H->g, H->axis, (const double2 *)psi_T, (double2 *)lam, nst, ldp, s))) return rc;
    const int64_t nseg = (nsteps + ckpt_every - 1) / ckpt_every;
    // per segment: recompute every step from the checkpoint keeping its
    // stage outputs (state k in states slot k, k >= 1; the last step's
    // output, the next checkpoint, goes to the unused slot 0), then the
    // adjoint steps backward over the kept stages
    for (int64_t seg = nseg - 1; seg >= 0; --seg) {
        const int64_t s0 = seg * ckpt_every, s1 = std::min(nsteps, s0 + ckpt_every);
        const char *ck = (const char *)ckpt_dev + (size_t)seg * bb;
        auto st = [&](int64_t k) -> char * { return k == 0 ? const_cast<char *>(ck) : states + k * bbr; };
        auto yk = [&](int64_t k, int j) -> char * { return ystore + (3 * k + j) * bbr; };
        for (int64_t k = 0; k < (keep ? s1 - s0 : s1 - s0 - 1); ++k) {
            void *y[3] = {yk(keep ? k : 0, 0), yk(keep ? k : 0, 1), yk(keep ? k : 0, 2)};
            void *next = k + 1 < s1 - s0 ? (void *)st(k + 1) : (void *)states;
            if ((rc = step_product(*H, st(k), y, next, nst, ldp, dt, 0.0, fields + s0 + k, sws, s))) return rc;
        }
        for (int64_t n = s1 - 1; n >= s0; --n) {
            const int64_t k = n - s0;
            if (!keep) {
                // this step's stage outputs again, into the one-step store
                void *y3[3] = {yk(0, 0), yk(0, 1), yk(0, 2)};
                if ((rc = step_product(*H, st(k), y3, nullptr, nst, ldp, dt, 0.0, fields + n, sws, s))) return rc;
            }
            const int64_t kk = keep ? k : 0;
            const void *y[4] = {st(k), yk(kk, 0), yk(kk, 1), yk(kk, 2)};
            if ((rc = adjoint_product_impl(*H, y, lam, nst, ldp, dt, 0.0, fields + n, gs + n, sws, rest, s)))
                return rc;
        }
    }
    return rsg_laser_grad(gs, nsteps, T, dt, ncoef, grad_dev, stream);
}

static int tile_compute(int32_t dtype) { return dtype == RSG_C128 ? 0 : 1; }

extern "C" int rsg_tile_candidates(int32_t dtype, rsg_tile *out, int32_t max, int32_t *count) {
    clear_error();
    RSG_REQUIRE(dtype == RSG_C128 || dtype == RSG_C64_MIXED, RSG_EDTYPE, "rsg_tile_candidates: bad dtype");
    RSG_REQUIRE(count && (max <= 0 || out), RSG_EINVAL, "rsg_tile_candidates: null output");
    const auto v = tile_candidates(tile_compute(dtype));
    *count = (int32_t)v.size();
    for (int32_t k = 0; k < max && k < (int32_t)v.size(); ++k)
        out[k] = rsg_tile{v[k].B, v[k].TX, v[k].TY, 0, v[k].PD, 0, 0, 0};
    return RSG_OK;
}

extern "C" int rsg_set_tile(rsg_ham_t H, int64_t nst, int32_t dtype, const rsg_tile *t) {
    clear_error();
    RSG_REQUIRE(H && t, RSG_EINVAL, "rsg_set_tile: null argument");
    RSG_REQUIRE(dtype == RSG_C128 || dtype == RSG_C64_MIXED, RSG_EDTYPE, "rsg_set_tile: bad dtype");
    RSG_REQUIRE(t->ZC >= 0, RSG_EINVAL, "rsg_set_tile: ZC must be >= 0");
    bool ok = false;
    const int pd = t->PD;
    for (const auto &c : tile_candidates(tile_compute(dtype)))
        ok = ok || (c.B == t->B && c.TX == t->TX && c.TY == t->TY && c.PD == pd);
    RSG_REQUIRE(ok, RSG_EUNSUPPORTED, "rsg_set_tile: %dx%dx%d (depth %d) is not a compiled tile shape", t->B,
                t->TX, t->TY, t->PD);
    RSG_REQUIRE(t->PT >= 0 && t->PT <= 64, RSG_EINVAL, "rsg_set_tile: PT must be in 0..64");
    RSG_REQUIRE(t->BO >= 0 && t->BO <= 64, RSG_EINVAL, "rsg_set_tile: BO must be in 0..64");
    RSG_REQUIRE(t->ZM >= 0 && t->ZM <= 2, RSG_EINVAL, "rsg_set_tile: ZM must be 0, 1 or 2");
    TileShape sh{t->B, t->TX, t->TY, t->ZC};
    sh.PD = pd;
    sh.PT = t->PT;
    sh.BO = t->BO;
    sh.ZM = t->ZM;
    H->tiles[std::make_pair(nst, tile_compute(dtype))] = sh;
    drop_graphs(H);
    return RSG_OK;
}

extern "C" int rsg_get_tile(rsg_ham_t H, int64_t nst, int32_t dtype, rsg_tile *t) {
    clear_error();
    RSG_REQUIRE(H && t, RSG_EINVAL, "rsg_get_tile: null argument");
    RSG_REQUIRE(dtype == RSG_C128 || dtype == RSG_C64_MIXED, RSG_EDTYPE, "rsg_get_tile: bad dtype");
    const TileShape s = H->tile_for(nst, tile_compute(dtype));
    *t = rsg_tile{s.B, s.TX, s.TY, s.ZC, s.PD, s.PT, s.BO, s.ZM};
    return RSG_OK;
}

// Times one Taylor stage (out = psi + c H psi into the workspace, psi
// untouched) for every compiled tile shape, z-chunk length, tile order,
// block order and z-march, re-times the six fastest with three times the
// launches, keeps the fastest for (nst, dtype) and reports it.
extern "C" int rsg_autotune(rsg_ham_t H, const void *psi, int64_t nst, int64_t ldp, int32_t dtype,
                            void *ws, size_t ws_bytes, int32_t reps, rsg_tile *best, double *best_ms,
                            void *stream) {
    clear_error();
    int rc = check_batch(H, psi, nst, ldp, "rsg_autotune");
    if (rc) return rc;
    RSG_REQUIRE(dtype == RSG_C128 || dtype == RSG_C64_MIXED, RSG_EDTYPE, "rsg_autotune: bad dtype");
    RSG_REQUIRE(nst > 0 && reps > 0, RSG_EINVAL, "rsg_autotune: need nst > 0 and reps > 0");
    RSG_REQUIRE(ws_bytes >= step_ws(*H, nst, ldp, dtype) - 256, RSG_ENOMEM, "rsg_autotune: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int cmp = tile_compute(dtype);
    const int wt = cmp;  // work-buffer type: complex64 for the mixed path
    Carve c(ws, ws_bytes);
    void *w1 = c.take(batch_bytes(nst, ldp, cmp ? 8 : 16));
    void *w2 = c.take(batch_bytes(nst, ldp, cmp ? 8 : 16));
    if (!c.ok) {
        set_error("rsg_autotune: workspace carve failed");
        return RSG_ENOMEM;
    }
    return guarded([&]() -> int {
        std::vector<int> zcs = {0};
        for (int z : {96, 64, 32})
            if (z < H->g->n[2]) zcs.push_back(z);
        // few tiles (small grid, few orbitals): short z-chunks for parallelism
        const int64_t small_tiles = (int64_t)((H->g->n[0] + 15) / 16) * ((H->g->n[1] + 7) / 8) * nst;
        if (small_tiles < 2048)
            for (int z : {16, 8, 4, 2, 1})
                if (z < H->g->n[2]) zcs.push_back(z);
        const std::vector<int> pts = {0, 1};
        const std::vector<int> bos = {0, 1, 2, 4};
        const int nzp = (int)(zcs.size() * pts.size()), nvar = nzp * (int)bos.size() * 3;  // x BO x ZM
        hipEvent_t e0, e1;
        RSG_CHECK_HIP(hipEventCreate(&e0));
        RSG_CHECK_HIP(hipEventCreate(&e1));
        // the two kinds of stage of a step: the first (reads psi once, its
        // centre tap is the base) and the middle ones (read a work buffer,
        // the same base, and write the other work buffer)
        StageArgs first;
        first.in = psi;
        first.base = psi;
        first.out = w1;
        first.in_t = 0;
        first.out_t = wt;
        first.compute = cmp;
        first.mode = 1;
        first.first = true;
        first.nst = nst;
        first.ldp = ldp;
        first.cim = -1e-3;
        StageArgs rest = first;
        rest.in = w1;
        rest.in_t = wt;
        rest.out = w2;
        // the middle stages of every step form read only their input
        rest.base = w1;
        rest.first = true;
        int err = RSG_OK;
        // the work buffer read by the other stages holds a real stage output
        if ((rc = launch_stencil(*H, first, default_shape(*H->g, nst, cmp), s))) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return rc;
        }
        // best of n timings of one stage with shape sh, after a warm-up
        // launch.  A stage shorter than 0.2 ms is timed as the mean of a
        // burst of 16 back-to-back launches, as the stages of a step or a
        // captured sequence run: alone, such a launch measures mostly its
        // own start-up, which back-to-back launches overlap.
        auto time_stage = [&](const StageArgs &a, const TileShape &sh, int n, double *tmin) -> int {
            *tmin = 1e300;
            int burst = 1;
            for (int r = 0; r <= n; ++r) {
                RSG_CHECK_HIP(hipEventRecord(e0, s));
                for (int k = 0; k < burst; ++k) {
                    const int q = launch_stencil(*H, a, sh, s);
                    if (q) return q;
                }
                RSG_CHECK_HIP(hipEventRecord(e1, s));
                RSG_CHECK_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                RSG_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (r == 0) {
                    if (ms < 0.2f) burst = 16;
                } else {
                    *tmin = std::min(*tmin, (double)ms / burst);
                }
            }
            return RSG_OK;
        };
        // phase 1 ranks by one of the other stages; phase 2 by the stencil
        // time of a whole step, first + 3 others
        auto time_shape = [&](const TileShape &sh, int n, double *t) -> int {
            return time_stage(rest, sh, n, t);
        };
        // (short stages: best of n bursts of 8 back-to-back stage sequences
        // first, rest, rest, rest, the order of a step's launches)
        auto time_step = [&](const TileShape &sh, int n, double *t) -> int {
            double t1 = 0, t2 = 0;
            int q = time_stage(first, sh, n, &t1);
            if (!q) q = time_stage(rest, sh, n, &t2);
            *t = t1 + 3.0 * t2;
            if (q || *t >= 0.8) return q;
            *t = 1e300;
            for (int r = 0; r < n; ++r) {
                RSG_CHECK_HIP(hipEventRecord(e0, s));
                for (int k = 0; k < 8 && !q; ++k) {
                    q = launch_stencil(*H, first, sh, s);
                    for (int j = 0; j < 3 && !q; ++j) q = launch_stencil(*H, rest, sh, s);
                }
                if (q) return q;
                RSG_CHECK_HIP(hipEventRecord(e1, s));
                RSG_CHECK_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                RSG_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
                *t = std::min(*t, (double)ms / 8);
            }
            return RSG_OK;
        };
        // phase 1: every candidate, reps launches each
        std::vector<std::pair<double, TileShape>> timed;
        for (const auto &cand : tile_candidates(cmp)) {
            for (int zpi = 0; zpi < nvar && !rc && !err; ++zpi) {
                const int zc = zcs[zpi % zcs.size()];
                TileShape sh = cand;
                sh.ZC = zc > 0 ? zc : H->g->n[2];
                sh.PT = pts[(zpi / zcs.size()) % pts.size()];
                sh.BO = bos[(zpi / nzp) % bos.size()];
                sh.ZM = zpi / (nzp * (int)bos.size());
                // chunks aligned in z need chunks, and are tried in row order
                // with the orbital slowest or in pairs only
                if (sh.ZM == 2 && (zc == 0 || sh.PT != 0 || (sh.BO != 1 && sh.BO != 2))) continue;
                if (!H->g->plan(sh, s, &err)) break;
                double t = 0;
                if ((rc = time_shape(sh, reps, &t))) break;
                timed.emplace_back(t, sh);
            }
            if (rc || err) break;
        }
        // phase 2: the few fastest again with more launches, so that shapes
        // within timing noise of each other are told apart
        double bt = 1e300;
        TileShape bs = default_shape(*H->g, nst, cmp);
        if (!rc && !err) {
            std::stable_sort(timed.begin(), timed.end(),
                             [](const std::pair<double, TileShape> &p, const std::pair<double, TileShape> &q) {
                                 return p.first < q.first;
                             });
            const size_t keep = std::min<size_t>(6, timed.size());
            for (size_t k = 0; k < keep && !rc; ++k) {
                double t = 0;
                if ((rc = time_step(timed[k].second, 3 * reps, &t))) break;
                if (t < bt) {
                    bt = t;
                    bs = timed[k].second;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (err) return err;
        if (rc) return rc;
        H->tiles[std::make_pair(nst, cmp)] = bs;
        drop_graphs(H);
        if (best) *best = rsg_tile{bs.B, bs.TX, bs.TY, bs.ZC, bs.PD, bs.PT, bs.BO, bs.ZM};
        if (best_ms) *best_ms = bt;
        return RSG_OK;
    });
}

// Key of a tuned tile in the cache file: everything the choice depends on
// (box shape and size, storage alignment, orbital count, precision, the
// kernel family in use, and the device).
static int tile_cache_key(const Ham &H, int64_t nst, int32_t dtype, std::string *key) {
    int dev = 0;
    hipDeviceProp_t prop;
    RSG_CHECK_HIP(hipGetDevice(&dev));
    RSG_CHECK_HIP(hipGetDeviceProperties(&prop, dev));
    const Grid &g = *H.g;
    char buf[512];
    snprintf(buf, sizeof buf, "box=%d dims=%dx%dx%d points=%lld slots=%lld align=%d nst=%lld dtype=%d cs=%d mask=%d dev=%s/%d",
             g.shape, g.n[0], g.n[1], g.n[2], (long long)g.npts, (long long)g.np, g.align, (long long)nst, dtype,
             H.complex_scaled() ? 1 : 0, H.mask ? 1 : 0, prop.gcnArchName, prop.multiProcessorCount);
    *key = buf;
    return RSG_OK;
}

extern "C" int rsg_autotune_cache(rsg_ham_t H, const void *psi, int64_t nst, int64_t ldp, int32_t dtype, void *ws,
                                  size_t ws_bytes, int32_t reps, const char *cache_path, rsg_tile *best,
                                  double *best_ms, int32_t *cached, void *stream) {
    clear_error();
    RSG_REQUIRE(H && cache_path, RSG_EINVAL, "rsg_autotune_cache: null argument");
    RSG_REQUIRE(dtype == RSG_C128 || dtype == RSG_C64_MIXED, RSG_EDTYPE, "rsg_autotune_cache: bad dtype");
    RSG_REQUIRE(nst > 0 && reps > 0, RSG_EINVAL, "rsg_autotune_cache: need nst > 0 and reps > 0");
    return guarded([&]() -> int {
        std::string key;
        int rc = tile_cache_key(*H, nst, dtype, &key);
        if (rc) return rc;
        if (cached) *cached = 0;
        // the last entry of this key wins
        bool found = false;
        rsg_tile t{};
        double ms = 0.0;
        if (FILE *f = std::fopen(cache_path, "r")) {
            char line[1024];
            while (std::fgets(line, sizeof line, f)) {
                char *bar = std::strchr(line, '|');
                if (!bar || (size_t)(bar - line) != key.size() + 1 || std::strncmp(line, key.c_str(), key.size()))
                    continue;
                rsg_tile u{};
                double m = 0.0;
                if (std::sscanf(bar + 1, " %d %d %d %d %d %d %d %d | %lf", &u.B, &u.TX, &u.TY, &u.ZC, &u.PD, &u.PT,
                                &u.BO, &u.ZM, &m) == 9) {
                    t = u;
                    ms = m;
                    found = true;
                }
            }
            std::fclose(f);
        }
        if (found && rsg_set_tile(H, nst, dtype, &t) == RSG_OK) {
            if (best) *best = t;
            if (best_ms) *best_ms = ms;
            if (cached) *cached = 1;
            return RSG_OK;
        }
        clear_error();  // a stale entry (a tile no longer compiled) is timed again
        rc = rsg_autotune(H, psi, nst, ldp, dtype, ws, ws_bytes, reps, &t, &ms, stream);
        if (rc) return rc;
        if (best) *best = t;
        if (best_ms) *best_ms = ms;
        FILE *f = std::fopen(cache_path, "a");
        RSG_REQUIRE(f, RSG_EINVAL, "rsg_autotune_cache: cannot append to %s", cache_path);
        std::fprintf(f, "%s | %d %d %d %d %d %d %d %d | %.17g\n", key.c_str(), t.B, t.TX, t.TY, t.ZC, t.PD, t.PT,
                     t.BO, t.ZM, ms);
        const bool ok = std::fclose(f) == 0;
        RSG_REQUIRE(ok, RSG_EINVAL, "rsg_autotune_cache: writing %s failed", cache_path);
        return RSG_OK;
    });
}

extern "C" int rsg_copy(const void *src, void *dst, size_t nbytes, void *stream) {
    clear_error();
    RSG_REQUIRE(nbytes % 16 == 0, RSG_EINVAL, "rsg_copy: size must be a multiple of 16");
    RSG_REQUIRE(nbytes == 0 || (src && dst), RSG_EINVAL, "rsg_copy: null pointer");
    RSG_REQUIRE((((uintptr_t)src | (uintptr_t)dst) & 15) == 0, RSG_EINVAL, "rsg_copy: unaligned pointer");
    if (nbytes == 0) return RSG_OK;
    const int64_t n16 = (int64_t)(nbytes / 16);
    int64_t nb = (n16 + 255) / 256;
    nb = std::min<int64_t>(nb, 256 * 16);
    timing_before((hipStream_t)stream);
    k_copy16<<<(unsigned)nb, 256, 0, (hipStream_t)stream>>>((const int4 *)src, (int4 *)dst, n16);
    timing_after((hipStream_t)stream);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

extern "C" int rsg_timing_enable(int32_t on) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = on != 0;
    return RSG_OK;
}

extern "C" int rsg_timing_query(int64_t *count, double *mean_ms, double *total_ms) {
    clear_error();
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        ev.swap(g_events);
    }
    double tot = 0.0;
    int64_t n = 0;
    int rc = RSG_OK;
    for (auto &p : ev) {
        float ms = 0.f;
        if (hipEventSynchronize(p.second) == hipSuccess && hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess) {
            tot += ms;
            ++n;
        } else {
            rc = RSG_EHIP;
        }
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    if (count) *count = n;
    if (total_ms) *total_ms = tot;
    if (mean_ms) *mean_ms = n ? tot / n : 0.0;
    if (rc) set_error("rsg_timing_query: event query failed");
    return rc;
}
