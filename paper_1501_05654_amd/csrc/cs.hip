// Eigenvalues of a complex-scaled Hamiltonian near given targets.
//
// Section "Complex scaling and resonances": H_theta is symmetric but not
// Hermitian; its bound states keep their energies, the continuum rotates by
// -2 theta and resonances appear as isolated eigenvalues eps - i Gamma/2.
// Matrix elements take no complex conjugation, so a state is normalised by
// h^3 sum x^2 = 1 and its energy is the symmetric Rayleigh quotient
// h^3 sum x (H x).
//
// Method: shifted inverse iteration, one orbital per target z_n: x <- (H -
// z_n)^{-1} x, solved with the library's QMR (H - z_n is complex symmetric),
// normalised in the bilinear form, lambda_n = x^T H x.  Converges to the
// eigenvalue nearest z_n at the rate |lambda_1 - z| / |lambda_2 - z|.
#include "rsg_internal.h"

#include <cmath>
#include <complex>
#include <vector>

namespace rsg {

namespace {

// x[n][i] = c_n y[n][i]
__global__ void __launch_bounds__(256) k_cs_scale(const double2 *__restrict__ y, double2 *__restrict__ x,
                                                  const double2 *__restrict__ c, int64_t np, int64_t ldp) {
    const int64_t n = blockIdx.y;
    const double2 cc = c[n];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 v = y[n * ldp + i];
        x[n * ldp + i] = make_double2(cc.x * v.x - cc.y * v.y, cc.x * v.y + cc.y * v.x);
    }
}

}  // namespace

}  // namespace rsg

using namespace rsg;

extern "C" size_t rsg_cs_eigs_workspace_bytes(rsg_ham_t H, int64_t nst, int64_t ldp) {
    if (!H || nst < 1 || ldp < 1) return 0;
    return 2 * rounded(batch_bytes(nst, ldp, 16)) + rounded(rsg_solve_workspace_bytes(H, RSG_SOLVE_QMR, nst, ldp)) +
           rounded(reduce_workspace_bytes(*H->g, nst)) + rounded(kb_workspace_bytes(*H, nst)) +
           2 * rounded(sizeof(double2) * nst) + 256;
}

extern "C" int rsg_cs_eigs(rsg_ham_t H, const double *target, void *psi, int64_t nst, int64_t ldp, int32_t max_outer,
                           double tol, int32_t qmr_maxiter, double qmr_tol, double *lambda, int32_t *outer_iters,
                           void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc = check_batch(H, psi, nst, ldp, "rsg_cs_eigs");
    if (rc) return rc;
    RSG_REQUIRE(nst >= 1 && nst <= 65535, RSG_ESHAPE, "rsg_cs_eigs: need 1 <= nst <= 65535");
    RSG_REQUIRE(target && lambda, RSG_EINVAL, "rsg_cs_eigs: null target or lambda");
    RSG_REQUIRE(max_outer >= 1 && qmr_maxiter >= 1 && tol >= 0 && qmr_tol >= 0 && std::isfinite(tol) &&
                    std::isfinite(qmr_tol),
                RSG_EINVAL, "rsg_cs_eigs: need max_outer, qmr_maxiter >= 1 and tolerances >= 0");
    for (int64_t n = 0; n < 2 * nst; ++n)
        RSG_REQUIRE(std::isfinite(target[n]), RSG_EINVAL, "rsg_cs_eigs: target not finite");
    const size_t bb = batch_bytes(nst, ldp, 16);
    Carve c(ws, ws_bytes);
    void *y = c.take(bb);
    void *hx = c.take(bb);
    const size_t sws = rsg_solve_workspace_bytes(H, RSG_SOLVE_QMR, nst, ldp);
    void *sw = c.take(sws);
    const size_t rb = reduce_workspace_bytes(*H->g, nst);
    void *R = c.take(rb);
    void *D = c.take(kb_workspace_bytes(*H, nst));
    double *red = static_cast<double *>(c.take(sizeof(double2) * nst));
    double2 *scale = static_cast<double2 *>(c.take(sizeof(double2) * nst));
    RSG_REQUIRE(c.ok, RSG_ENOMEM, "rsg_cs_eigs: workspace too small (%zu < %zu bytes)", ws_bytes,
                rsg_cs_eigs_workspace_bytes(H, nst, ldp));
    hipStream_t s = (hipStream_t)stream;
    const int64_t np = H->g->np;
    return guarded([&]() -> int {
        std::vector<double> shift(2 * nst), hred(2 * nst);
        std::vector<double2> hscale(nst);
        std::vector<std::complex<double>> lam(nst), prev(nst, std::complex<double>(NAN, NAN));
        for (int64_t n = 0; n < nst; ++n) {
            shift[2 * n] = -target[2 * n];
            shift[2 * n + 1] = -target[2 * n + 1];
        }
        const dim3 sg((unsigned)std::min<int64_t>(std::max<int64_t>((np + 255) / 256, 1), 1024), (unsigned)nst);
        auto normalise = [&](const void *src) -> int {
            // psi = src / sqrt(h^3 src^T src)
            int r = launch_reduce(*H->g, 3, 0, (const double2 *)src, (const double2 *)src, nst, ldp, red, R, rb, s);
            if (r) return r;
            RSG_CHECK_HIP(hipMemcpyAsync(hred.data(), red, sizeof(double) * 2 * nst, hipMemcpyDeviceToHost, s));
            RSG_CHECK_HIP(hipStreamSynchronize(s));
            for (int64_t n = 0; n < nst; ++n) {
                const std::complex<double> q(hred[2 * n], hred[2 * n + 1]);
                RSG_REQUIRE(std::abs(q) > 0 && std::isfinite(std::abs(q)), RSG_EINVAL,
                            "rsg_cs_eigs: orbital %lld has zero bilinear norm", (long long)n);
                const std::complex<double> f = 1.0 / std::sqrt(q);
                hscale[n] = make_double2(f.real(), f.imag());
            }
            RSG_CHECK_HIP(hipMemcpyAsync(scale, hscale.data(), sizeof(double2) * nst, hipMemcpyHostToDevice, s));
            k_cs_scale<<<sg, 256, 0, s>>>((const double2 *)src, (double2 *)psi, scale, np, ldp);
            RSG_CHECK_HIP(hipGetLastError());
            // hscale must outlive the copy above
            RSG_CHECK_HIP(hipStreamSynchronize(s));
            return RSG_OK;
        };
        int r;
        if ((r = normalise(psi))) return r;
        int done = 0;
        for (int it = 0; it < max_outer; ++it) {
            // y = (H - z)^{-1} psi
            RSG_CHECK_HIP(hipMemsetAsync(y, 0, bb, s));
            r = rsg_shifted_solve(H, shift.data(), psi, y, nst, ldp, RSG_SOLVE_QMR, qmr_tol, qmr_maxiter, 10,
                                  nullptr, nullptr, nullptr, sw, sws, s);
            if (r) return r;
            if ((r = normalise(y))) return r;
            // lambda = h^3 psi^T H psi
            if ((r = hpsi_impl(*H, psi, hx, nst, ldp, 0.0, nullptr, D, s))) return r;
            if ((r = launch_reduce(*H->g, 3, 0, (const double2 *)psi, (const double2 *)hx, nst, ldp, red, R, rb, s)))
                return r;
            RSG_CHECK_HIP(hipMemcpyAsync(hred.data(), red, sizeof(double) * 2 * nst, hipMemcpyDeviceToHost, s));
            RSG_CHECK_HIP(hipStreamSynchronize(s));
            bool conv = true;
            for (int64_t n = 0; n < nst; ++n) {
                lam[n] = std::complex<double>(hred[2 * n], hred[2 * n + 1]);
                if (!(std::abs(lam[n] - prev[n]) <= tol * std::max(1.0, std::abs(lam[n])))) conv = false;
                prev[n] = lam[n];
            }
            done = it + 1;
            if (conv) break;
        }
        for (int64_t n = 0; n < nst; ++n) {
            lambda[2 * n] = lam[n].real();
            lambda[2 * n + 1] = lam[n].imag();
            if (outer_iters) outer_iters[n] = done;
        }
        return RSG_OK;
    });
}
