// Projector terms of a fused two-factor pass.
//
// With H = L + N (L local: kinetic, V, dipole; N the separable projectors,
// N y = sum_a P_a E_a D_a(y), D_a(y) = h^3 P_a^T y on the support S_a), the
// fused z-march computes w = (1 + cb L)(1 + ca L) y0.  The two factors of H
// differ from it only near the supports:
//   y1 = (1 + ca L) y0 + s1,             s1 = ca N y0 (zero outside S),
//   (1 + cb H) y1 = w + s1 + cb L s1 + cb N y1,
// and L s1 vanishes outside S dilated by the stencil star (SS).  So:
//   1. D0 = D(y0)                       (gather over the supports)
//   2. s1 = ca P E D0 on S               (scatter into a compact array)
//   3. y1 = y0 + ca L y0 + s1 on S       (point-list stencil)
//   4. D1 = D(y1)                        (gather from the compact array)
//   5. w += s1 + cb L s1 on SS           (point-list stencil of s1)
//   6. w += cb P E D1                    (scatter over the supports)
// Every step reads or writes only the supports and their star (a few per
// cent of the grid on the benchmark sphere), and the result equals the two
// single-factor stages up to rounding.
#include "rsg_internal.h"

#include <algorithm>

namespace rsg {

namespace {

constexpr double C0 = -205.0 / 72.0, C1 = 8.0 / 5.0, C2 = -1.0 / 5.0, C3 = 8.0 / 315.0, C4 = -1.0 / 560.0;

struct PtArgs {
    const double2 *y0;   // full-grid input [nst][ldp]
    const double2 *s1;   // compact s1 [nst][nS]
    double2 *y1;         // compact y1 [nst][nS]
    double2 *w;          // full-grid output [nst][ldp]
    const int32_t *slot, *nb, *spos;
    const double *V;
    const int32_t *ijk;
    const double *field_dev;
    int64_t npt, nS, ldp;
    double field, kin_h2, h, off;
    int32_t axis;
    double cr, ci;
};

__device__ __forceinline__ double axis_coord(const PtArgs &a, int slot) {
    return a.h * ((double)a.ijk[3 * slot + a.axis] - a.off);
}

// y1 = y0 + c (kin/h^2 Lap y0 + (V + E x) y0) + s1 at the points of S.
// Neighbour k of point i: nb[k * npt + i], k = 8 axis + 2 (m - 1) + side.
__global__ void __launch_bounds__(256) k_pts_first(PtArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.npt) return;
    const int64_t n = blockIdx.y;
    const double2 *y0 = a.y0 + n * a.ldp;
    const int slot = a.slot[i];
    const double2 q = y0[slot];
    const double c[5] = {C0, C1, C2, C3, C4};
    double lr = 3.0 * C0 * q.x, li = 3.0 * C0 * q.y;
#pragma unroll
    for (int m = 1; m <= 4; ++m)
#pragma unroll
        for (int ax = 0; ax < 3; ++ax)
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int j = a.nb[(int64_t)(8 * ax + 2 * (m - 1) + side) * a.npt + i];
                if (j >= 0) {
                    const double2 v = y0[j];
                    lr += c[m] * v.x;
                    li += c[m] * v.y;
                }
            }
    double v = a.V[slot];
    if (a.axis >= 0) v += (a.field_dev ? *a.field_dev : a.field) * axis_coord(a, slot);
    const double hr = a.kin_h2 * lr + v * q.x, hi = a.kin_h2 * li + v * q.y;
    const double2 s = a.s1[n * a.nS + i];
    a.y1[n * a.nS + i] = make_double2(q.x + (a.cr * hr - a.ci * hi) + s.x, q.y + (a.cr * hi + a.ci * hr) + s.y);
}

// w += s1 + c (kin/h^2 Lap s1 + (V + E x) s1) at the points of SS (s1 zero
// outside S; neighbours given as positions in S, -1 if none).
__global__ void __launch_bounds__(256) k_pts_second(PtArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.npt) return;
    const int64_t n = blockIdx.y;
    const double2 *s1 = a.s1 + n * a.nS;
    const int slot = a.slot[i], sp = a.spos[i];
    const double2 q = sp >= 0 ? s1[sp] : make_double2(0.0, 0.0);
    const double c[5] = {C0, C1, C2, C3, C4};
    double lr = 3.0 * C0 * q.x, li = 3.0 * C0 * q.y;
#pragma unroll
    for (int m = 1; m <= 4; ++m)
#pragma unroll
        for (int ax = 0; ax < 3; ++ax)
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int j = a.nb[(int64_t)(8 * ax + 2 * (m - 1) + side) * a.npt + i];
                if (j >= 0) {
                    const double2 v = s1[j];
                    lr += c[m] * v.x;
                    li += c[m] * v.y;
                }
            }
    double v = a.V[slot];
    if (a.axis >= 0) v += (a.field_dev ? *a.field_dev : a.field) * axis_coord(a, slot);
    const double hr = a.kin_h2 * lr + v * q.x, hi = a.kin_h2 * li + v * q.y;
    double2 *w = a.w + n * a.ldp + slot;
    const double2 o = *w;
    *w = make_double2(o.x + q.x + (a.cr * hr - a.ci * hi), o.y + q.y + (a.cr * hi + a.ci * hr));
}

__global__ void k_zero2(double2 *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_double2(0.0, 0.0);
}

template <class T>
int upload_vec(T **dst, const std::vector<T> &v) {
    RSG_CHECK_HIP(hipMalloc(dst, sizeof(T) * std::max<size_t>(v.size(), 1)));
    if (!v.empty()) RSG_CHECK_HIP(hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return RSG_OK;
}

}  // namespace

int build_support_tables(Ham &H, const std::vector<int32_t> &idx_padded) {
    const Grid &g = *H.g;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    std::vector<int32_t> ijk((size_t)3 * g.np);
    RSG_CHECK_HIP(hipMemcpy(ijk.data(), g.ijk, sizeof(int32_t) * ijk.size(), hipMemcpyDeviceToHost));
    auto slot_of = [&](int x, int y, int z) -> int32_t {
        if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) return -1;
        const int2 r = g.rows_host[(size_t)z * ny + y];
        const int a = r.y & 0xffff, b = (r.y >> 16) & 0xffff;
        return (x >= a && x < b) ? r.x + x : -1;
    };
    // S: every listed support point (the padded entries repeat a real one)
    std::vector<int32_t> S;
    for (int a = 0; a < H.natoms; ++a)
        for (int64_t k = 0; k < H.kb_len[a]; ++k) S.push_back(idx_padded[H.kb_off[a] + k]);
    std::sort(S.begin(), S.end());
    S.erase(std::unique(S.begin(), S.end()), S.end());
    const int64_t nS = (int64_t)S.size();
    std::vector<int32_t> pos(g.np, -1);
    for (int64_t i = 0; i < nS; ++i) pos[S[i]] = (int32_t)i;
    auto star = [&](int32_t slot, int k) -> int32_t {
        const int ax = k / 8, m = (k % 8) / 2 + 1, sg = (k % 2) ? 1 : -1;
        int c[3] = {ijk[3 * (size_t)slot], ijk[3 * (size_t)slot + 1], ijk[3 * (size_t)slot + 2]};
        c[ax] += sg * m;
        return slot_of(c[0], c[1], c[2]);
    };
    std::vector<int32_t> snb((size_t)24 * nS);
    std::vector<int32_t> SS(S);
    for (int64_t i = 0; i < nS; ++i)
        for (int k = 0; k < 24; ++k) {
            const int32_t j = star(S[i], k);
            snb[(size_t)k * nS + i] = j;
            if (j >= 0) SS.push_back(j);
        }
    std::sort(SS.begin(), SS.end());
    SS.erase(std::unique(SS.begin(), SS.end()), SS.end());
    const int64_t nSS = (int64_t)SS.size();
    std::vector<int32_t> ssp(nSS), ssnb((size_t)24 * nSS);
    for (int64_t i = 0; i < nSS; ++i) {
        ssp[i] = pos[SS[i]];
        for (int k = 0; k < 24; ++k) {
            const int32_t j = star(SS[i], k);
            ssnb[(size_t)k * nSS + i] = j >= 0 ? pos[j] : -1;
        }
    }
    std::vector<int32_t> cidx(idx_padded.size());
    for (size_t e = 0; e < idx_padded.size(); ++e) cidx[e] = pos[idx_padded[e]] >= 0 ? pos[idx_padded[e]] : 0;
    H.nS = nS;
    H.nSS = nSS;
    int rc;
    if ((rc = upload_vec(&H.sup_slot, S))) return rc;
    if ((rc = upload_vec(&H.sup_nb, snb))) return rc;
    if ((rc = upload_vec(&H.kb_cidx, cidx))) return rc;
    if ((rc = upload_vec(&H.ss_slot, SS))) return rc;
    if ((rc = upload_vec(&H.ss_s, ssp))) return rc;
    if ((rc = upload_vec(&H.ss_nb, ssnb))) return rc;
    return RSG_OK;
}

size_t fused_projector_ws(const Ham &H, int64_t nst) {
    if (H.natoms == 0) return 0;
    return rounded(kb_workspace_bytes(H, nst)) + 2 * rounded((size_t)nst * (size_t)H.nS * 16) + 256;
}

int fused_projector_fix(const Ham &H, const FusedArgs &f, void *ws, size_t ws_bytes, hipStream_t s) {
    if (H.natoms == 0 || f.nst == 0 || H.nS == 0) return RSG_OK;
    Carve c(ws, ws_bytes);
    void *D = c.take(kb_workspace_bytes(H, f.nst));
    double2 *s1 = (double2 *)c.take((size_t)f.nst * H.nS * 16);
    double2 *y1 = (double2 *)c.take((size_t)f.nst * H.nS * 16);
    if (!c.ok) {
        set_error("fused step: projector workspace too small (%zu < %zu)", ws_bytes, fused_projector_ws(H, f.nst));
        return RSG_ENOMEM;
    }
    const Grid &g = *H.g;
    int rc;
    // 1-2: D0, then s1 = ca P E D0 on S
    if ((rc = launch_kb_gather(H, f.in, 0, 0, f.nst, f.ldp, D, s))) return rc;
    const int64_t ns1 = f.nst * H.nS;
    k_zero2<<<(unsigned)std::min<int64_t>((ns1 + 255) / 256, 4096), 256, 0, s>>>(s1, ns1);
    if ((rc = launch_kb_scatter(H, s1, 0, 0, f.nst, H.nS, D, f.ca.real(), f.ca.imag(), nullptr, s, H.kb_cidx)))
        return rc;
    PtArgs a;
    a.y0 = (const double2 *)f.in;
    a.s1 = s1;
    a.y1 = y1;
    a.w = (double2 *)f.out;
    a.V = H.V;
    a.ijk = g.ijk;
    a.field_dev = f.field_dev;
    a.nS = H.nS;
    a.ldp = f.ldp;
    a.field = f.field;
    a.kin_h2 = H.kin / (g.h * g.h);
    a.h = g.h;
    a.axis = H.axis;
    a.off = H.axis >= 0 ? 0.5 * (double)(g.n[H.axis] - 1) : 0.0;
    // 3: y1 on S
    a.slot = H.sup_slot;
    a.nb = H.sup_nb;
    a.spos = nullptr;
    a.npt = H.nS;
    a.cr = f.ca.real();
    a.ci = f.ca.imag();
    k_pts_first<<<dim3((unsigned)((H.nS + 255) / 256), (unsigned)f.nst), 256, 0, s>>>(a);
    // 4: D1 from the compact y1
    if ((rc = launch_kb_gather(H, y1, 0, 0, f.nst, H.nS, D, s, H.kb_cidx))) return rc;
    // 5: w += s1 + cb L s1 on SS
    a.slot = H.ss_slot;
    a.nb = H.ss_nb;
    a.spos = H.ss_s;
    a.npt = H.nSS;
    a.cr = f.cb.real();
    a.ci = f.cb.imag();
    k_pts_second<<<dim3((unsigned)((H.nSS + 255) / 256), (unsigned)f.nst), 256, 0, s>>>(a);
    RSG_CHECK_HIP(hipGetLastError());
    // 6: w += cb P E D1
    return launch_kb_scatter(H, f.out, 0, 0, f.nst, f.ldp, D, f.cb.real(), f.cb.imag(), nullptr, s);
}

}  // namespace rsg
