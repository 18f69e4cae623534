// Separable non-local projectors on MFMA.
//
//   V_nl psi_n = sum_a sum_i p_i^a E_i^a D[a][i][n],
//   D[a][i][n] = h^3 sum_{r in S_a} p_i^a(r) psi_n(r)
//
// The non-local pseudopotential and its projectors are the electron-ion
// term named in section "Magnetic response and gauge invariance in
// real-space grids"; the separable form with four real projectors per atom
// is this library's reading.  Both halves are dense contractions:
//
//   gather : D^T[cols x 4] = psi^T[cols x |S_a|] * P[|S_a| x 4]
//   scatter: Y[|S_a| x cols] += P[|S_a| x 4] * F[4 x cols],  F = c E D
//
// where cols are the 2*nst real columns (re and im of each orbital).  The
// batch is orbital-major: real column col of point r sits at
// (col / 2) * ldo + 2 r + col % 2 (in reals), ldo = 2 ldp.
// Both run on v_mfma_{f64,f32}_16x16x4: the gather puts 16 columns on M,
// 4 support points on K and the 4 projectors on N (zero-padded to 16); the
// scatter puts 16 support points on M, the 4 projectors on K and 16
// columns on N, which fills the instruction exactly.
//
// MFMA operand layout (lane l of a wave of 64), measured on gfx950:
//   A[i][k] in lane i + 16k, B[k][j] in lane j + 16k;
//   accumulator element r of lane l holds D[i][j] with j = l % 16 and
//     i = l/16 + 4r      for v_mfma_f64_16x16x4f64,
//     i = 4(l/16) + r    for v_mfma_f32_16x16x4f32.
//
// Supports are padded to a multiple of 16 entries with p = 0 (and a valid
// index); padded entries contribute zero and are never written.  Atoms whose
// supports overlap are scattered in different launches (colours), so no two
// lanes of one launch update the same point: the result is deterministic
// without atomics.
#include "rsg_internal.h"

#include <algorithm>

namespace rsg {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <class T> struct V4;
template <> struct V4<double> { using type = d4_t; };
template <> struct V4<float> { using type = f4_t; };

// Row of the accumulator element r held by lane group hi = l / 16.
__device__ __forceinline__ int acc_row(double, int hi, int r) { return hi + 4 * r; }
__device__ __forceinline__ int acc_row(float, int hi, int r) { return 4 * hi + r; }

__device__ __forceinline__ d4_t mfma16(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma16(float a, float b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Gather for one (atom, 16-column tile, support chunk): the support of 4-entry
// groups is cut into nchunk contiguous chunks; the GW waves of the workgroup
// split its chunk (wave w takes groups w, w+GW, ... of the chunk; each wave
// accumulates its groups in ascending order) and the partial products are
// added in wave order.  With one chunk the result goes to D scaled by h^3;
// with several, each chunk's sum goes to the partial buffer P and
// k_kb_gather_sum adds the chunks in order.  Either way the result does not
// depend on timing.  The group loop issues the index loads of GU groups,
// then their data loads, then the MFMAs, so GU gathers are in flight per
// wave.
constexpr int GW = 16;  // waves per gather workgroup
constexpr int GU = 4;   // groups in flight per wave
template <class Tin, class Tc>
__device__ __forceinline__ void gather_tile(const Tin *__restrict__ in, int64_t ldo, int64_t ncols,
                                            const int4 at, int a, int ct,
                                            const int32_t *__restrict__ idx,
                                            const Tc *__restrict__ p, Tc h3, Tc *__restrict__ D,
                                            Tc (*red)[64][4], int chunk = 0, int nchunk = 1,
                                            Tc *__restrict__ P = nullptr) {
    using V = typename V4<Tc>::type;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int lo = l & 15, hi = l >> 4;
    const int64_t col = (int64_t)ct * 16 + lo;
    const bool cok = col < ncols;
    const Tin *inc = in + (cok ? (col >> 1) * ldo + (col & 1) : 0);
    V acc = {0, 0, 0, 0};
    const int ngall = at.y >> 2;
    const int per = (ngall + nchunk - 1) / nchunk;
    const int g0 = min(ngall, chunk * per);
    const int ngroups = min(ngall, g0 + per);
    int gq = g0 + w;
    for (; gq + (GU - 1) * GW < ngroups; gq += GU * GW) {
        int64_t e[GU];
        int32_t ix[GU];
        Tc bv[GU], av[GU];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            e[u] = (int64_t)at.x + 4 * (gq + u * GW) + hi;
            ix[u] = idx[e[u]];
            bv[u] = lo < 4 ? p[e[u] * 4 + lo] : (Tc)0;
        }
#pragma unroll
        for (int u = 0; u < GU; ++u) av[u] = cok ? (Tc)inc[2 * (int64_t)ix[u]] : (Tc)0;
#pragma unroll
        for (int u = 0; u < GU; ++u) acc = mfma16(av[u], bv[u], acc);
    }
    for (; gq < ngroups; gq += GW) {
        const int64_t e = (int64_t)at.x + 4 * gq + hi;
        const Tc av = cok ? (Tc)inc[2 * (int64_t)idx[e]] : (Tc)0;
        const Tc bv = lo < 4 ? p[e * 4 + lo] : (Tc)0;
        acc = mfma16(av, bv, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) red[w][l][r] = acc[r];
    __syncthreads();
    if (w == 0 && lo < 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Tc v = red[0][l][r];
#pragma unroll
            for (int k = 1; k < GW; ++k) v += red[k][l][r];
            const int64_t c = (int64_t)ct * 16 + acc_row(Tc(0), hi, r);
            if (c < ncols) {
                if (nchunk == 1)
                    D[((int64_t)a * 4 + lo) * ncols + c] = h3 * v;
                else
                    P[(((int64_t)a * 4 + lo) * nchunk + chunk) * ncols + c] = v;
            }
        }
    }
}

// blockIdx.x = atom, blockIdx.y = tile of 16 real columns, blockIdx.z =
// support chunk (gridDim.z chunks).
template <class Tin, class Tc>
__global__ void __launch_bounds__(GW * 64) k_kb_gather(const Tin *__restrict__ in, int64_t ldo,
                                                       int64_t ncols, const int4 *__restrict__ atoms,
                                                       const int32_t *__restrict__ idx,
                                                       const Tc *__restrict__ p, Tc h3,
                                                       Tc *__restrict__ D, Tc *__restrict__ P) {
    __shared__ Tc red[GW][64][4];
    gather_tile<Tin, Tc>(in, ldo, ncols, atoms[blockIdx.x], blockIdx.x, blockIdx.y, idx, p, h3, D, red,
                         (int)blockIdx.z, (int)gridDim.z, P);
}

// D[a][i][c] = h3 * sum over chunks k = 0, 1, ... of P[a][i][k][c].
template <class Tc>
__global__ void __launch_bounds__(256) k_kb_gather_sum(const Tc *__restrict__ P, Tc *__restrict__ D,
                                                       int64_t nrows, int nchunk, int64_t ncols, Tc h3) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nrows * ncols) return;
    const int64_t row = t / ncols, c = t - row * ncols;
    const Tc *q = P + row * nchunk * ncols + c;
    // loads of 8 chunks in flight, added in chunk order
    Tc v = q[0];
    int k = 1;
    for (; k + 8 <= nchunk; k += 8) {
        Tc x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = q[(int64_t)(k + u) * ncols];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += x[u];
    }
    for (; k < nchunk; ++k) v += q[(int64_t)k * ncols];
    D[row * ncols + c] = h3 * v;
}


// Scatter for one (16-entry support tile, 16-column tile), one wave.
template <class Tout, class Tc>
__device__ __forceinline__ void scatter_tile(Tout *__restrict__ out, int64_t ldo, int64_t ncols,
                                             const int2 itm, const int4 at, int ct,
                                             const int32_t *__restrict__ idx,
                                             const Tc *__restrict__ p,
                                             const double *__restrict__ E,
                                             const Tc *__restrict__ D, double cre, double cim,
                                             const double *__restrict__ mask, Tc (*buf)[17]) {
    using V = typename V4<Tc>::type;
    const int l = threadIdx.x & 63;
    const int lo = l & 15, hi = l >> 4;
    const Tc av = p[((int64_t)itm.y + lo) * 4 + hi];
    const int64_t col = (int64_t)ct * 16 + lo;
    Tc bv = 0;
    if (col < ncols) {
        const int64_t n = col >> 1;
        const double dre = (double)D[((int64_t)itm.x * 4 + hi) * ncols + 2 * n];
        const double dim = (double)D[((int64_t)itm.x * 4 + hi) * ncols + 2 * n + 1];
        const double e = E[itm.x * 4 + hi];
        bv = (Tc)((col & 1) ? e * (cre * dim + cim * dre) : e * (cre * dre - cim * dim));
    }
    V zero = {0, 0, 0, 0};
    const V acc = mfma16(av, bv, zero);
    // the 16 x 16 tile (support entry x column) through this wave's LDS
    // slice, so that each lane then adds one complex value: a wave covers
    // 16 consecutive entries of 4 orbitals per pass (256-byte runs where the
    // support's points are consecutive)
#pragma unroll
    for (int r = 0; r < 4; ++r) buf[acc_row(Tc(0), hi, r)][lo] = acc[r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int64_t end = (int64_t)at.x + at.z;
    const int el = l & 15;
    const int64_t e = (int64_t)itm.y + el;
    const int64_t pt = e < end ? idx[e] : 0;
    const double m = (mask && e < end) ? mask[pt] : 1.0;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        const int o = (l >> 4) + 4 * pass;  // orbital within the column tile
        const int64_t c = (int64_t)ct * 16 + 2 * o;
        if (e < end && c < ncols) {
            Tout *dst = out + (c >> 1) * ldo + 2 * pt;
            const double are = (double)buf[el][2 * o], aim = (double)buf[el][2 * o + 1];
            const double addr = mask ? m * are : are, addi = mask ? m * aim : aim;
            dst[0] = (Tout)((double)dst[0] + addr);
            dst[1] = (Tout)((double)dst[1] + addi);
        }
    }
}

// One wave per (16-entry support tile, 16-column tile).
template <class Tout, class Tc>
__global__ void __launch_bounds__(256) k_kb_scatter(Tout *__restrict__ out, int64_t ldo, int64_t ncols,
                                                    const int2 *__restrict__ items, int32_t nitems,
                                                    const int4 *__restrict__ atoms,
                                                    const int32_t *__restrict__ idx,
                                                    const Tc *__restrict__ p,
                                                    const double *__restrict__ E,
                                                    const Tc *__restrict__ D, double cre,
                                                    double cim, const double *__restrict__ mask) {
    __shared__ Tc buf[4][16][17];  // one 16 x 16 tile per wave (padded rows)
    const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= nitems) return;
    const int2 itm = items[item];  // {atom, first entry}
    scatter_tile<Tout, Tc>(out, ldo, ncols, itm, atoms[itm.x], blockIdx.y, idx, p, E, D, cre, cim, mask,
                           buf[threadIdx.x >> 6]);
}

// Batched forms over many systems (FP64): item {system, atom, column tile}
// for the gather, {system, atom, first entry, column tile} for the scatter.
__global__ void __launch_bounds__(GW * 64) k_kb_gather_batch(const KbSys *__restrict__ sys,
                                                             const int4 *__restrict__ items) {
    __shared__ double red[GW][64][4];
    const int4 it = items[blockIdx.x];
    const KbSys &s = sys[it.x];
    gather_tile<double, double>(s.in, s.ldo, s.ncols, s.atoms[it.y], it.y, it.z, s.idx, s.p, s.h3, s.D,
                                red, it.w, s.nchunk, s.P);
}

// Same sum as k_kb_gather_sum, one workgroup per {system, block of 256 D
// entries}.
__global__ void __launch_bounds__(256) k_kb_gather_sum_batch(const KbSys *__restrict__ sys,
                                                             const int2 *__restrict__ items) {
    const int2 it = items[blockIdx.x];
    const KbSys &s = sys[it.x];
    const int64_t ncols = s.ncols, nrows = (int64_t)s.natoms * 4;
    const int64_t t = (int64_t)it.y * 256 + threadIdx.x;
    if (t >= nrows * ncols) return;
    const int64_t row = t / ncols, c = t - row * ncols;
    const int nchunk = s.nchunk;
    const double *q = s.P + row * nchunk * ncols + c;
    double v = q[0];
    int k = 1;
    for (; k + 8 <= nchunk; k += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = q[(int64_t)(k + u) * ncols];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += x[u];
    }
    for (; k < nchunk; ++k) v += q[(int64_t)k * ncols];
    s.D[row * ncols + c] = s.h3 * v;
}

__global__ void __launch_bounds__(256) k_kb_scatter_batch(const KbSys *__restrict__ sys,
                                                          const int4 *__restrict__ items, int32_t nitems,
                                                          double cre, double cim) {
    __shared__ double buf[4][16][17];  // one 16 x 16 tile per wave (padded rows)
    const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (item >= nitems) return;
    const int4 it = items[item];
    const KbSys &s = sys[it.x];
    scatter_tile<double, double>(s.out, s.ldo, s.ncols, make_int2(it.y, it.z), s.atoms[it.y], it.w, s.idx,
                                 s.p, s.E, s.D, cre, cim, nullptr, buf[threadIdx.x >> 6]);
}

}  // namespace

// Support chunks per (atom, column tile): enough workgroups to fill the chip
// when there are few atoms or few orbitals, each chunk at least 8 GW groups
// of 4 support entries of the smallest support (8 groups per wave: with
// fewer, a batch of many small systems ran tens of thousands of nearly
// empty gather workgroups).  The count depends on the system alone, so a
// system gives the same bits alone or in a batch.
int gather_chunks(const Ham &H, int64_t nst) {
    if (H.natoms == 0 || nst == 0) return 1;
    int64_t min_groups = INT64_MAX;
    for (int32_t a = 0; a < H.natoms; ++a) min_groups = std::min(min_groups, (H.kb_off[a + 1] - H.kb_off[a]) / 4);
    const int64_t tiles = (int64_t)H.natoms * ((2 * nst + 15) / 16);
    const int64_t want = (512 + tiles - 1) / tiles;
    const int64_t cap = std::max<int64_t>(1, min_groups / (8 * GW));
    return (int)std::max<int64_t>(1, std::min<int64_t>(std::min(want, cap), 64));
}

size_t gather_partials_offset(const Ham &H, int64_t nst) {
    const size_t dbytes = (size_t)H.natoms * 4 * 2 * (size_t)nst * sizeof(double);
    return (dbytes + 255) / 256 * 256;
}

// D [natoms][4][2 nst] plus, when the support is split, the chunk partials
// [natoms][4][nchunk][2 nst] behind it (sized for FP64 in every path).
size_t kb_workspace_bytes(const Ham &H, int64_t nst) {
    const size_t d = (size_t)H.natoms * 4 * 2 * (size_t)nst * sizeof(double);
    const int nchunk = gather_chunks(H, nst);
    return nchunk > 1 ? 2 * ((d + 255) / 256 * 256) + (size_t)nchunk * d : d;
}

int launch_kb_gather(const Ham &H, const void *in, int in_t, int compute, int64_t nst, int64_t ldp,
                     void *D, hipStream_t s) {
    if (H.natoms == 0 || nst == 0) return RSG_OK;
    const int64_t ncols = 2 * nst;
    const int nchunk = gather_chunks(H, nst);
    const dim3 grid((unsigned)H.natoms, (unsigned)((ncols + 15) / 16), (unsigned)nchunk);
    const double h3 = H.g->h * H.g->h * H.g->h;
    // the partials start at the first 256-byte boundary after D (FP64 size)
    void *P = nchunk > 1 ? (void *)((char *)D + gather_partials_offset(H, nst)) : nullptr;
    const int64_t nrows = (int64_t)H.natoms * 4;
    const unsigned sblk = (unsigned)((nrows * ncols + 255) / 256);
    if (compute == 0) {
        if (in_t != 0) return RSG_EUNSUPPORTED;
        k_kb_gather<double, double><<<grid, GW * 64, 0, s>>>((const double *)in, 2 * ldp, ncols,
                                                        H.gather_items, H.kb_idx, H.kb_p, h3,
                                                        (double *)D, (double *)P);
        if (nchunk > 1)
            k_kb_gather_sum<double><<<sblk, 256, 0, s>>>((const double *)P, (double *)D, nrows, nchunk, ncols, h3);
    } else {
        if (in_t == 0)
            k_kb_gather<double, float><<<grid, GW * 64, 0, s>>>((const double *)in, 2 * ldp, ncols,
                                                           H.gather_items, H.kb_idx, H.kb_p32,
                                                           (float)h3, (float *)D, (float *)P);
        else
            k_kb_gather<float, float><<<grid, GW * 64, 0, s>>>((const float *)in, 2 * ldp, ncols,
                                                          H.gather_items, H.kb_idx, H.kb_p32,
                                                          (float)h3, (float *)D, (float *)P);
        if (nchunk > 1)
            k_kb_gather_sum<float><<<sblk, 256, 0, s>>>((const float *)P, (float *)D, nrows, nchunk, ncols,
                                                        (float)h3);
    }
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

int launch_kb_scatter(const Ham &H, void *out, int out_t, int compute, int64_t nst, int64_t ldp,
                      const void *D, double cre, double cim, const double *mask, hipStream_t s) {
    if (H.natoms == 0 || nst == 0) return RSG_OK;
    const int64_t ncols = 2 * nst;
    for (size_t c = 0; c < H.scatter_items.size(); ++c) {
        const int32_t n = H.scatter_counts[c];
        if (n == 0) continue;
        const dim3 grid((unsigned)((n + 3) / 4), (unsigned)((ncols + 15) / 16));
        if (compute == 0) {
            if (out_t != 0) return RSG_EUNSUPPORTED;
            k_kb_scatter<double, double><<<grid, 256, 0, s>>>(
                (double *)out, 2 * ldp, ncols, H.scatter_items[c], n, H.gather_items, H.kb_idx,
                H.kb_p, H.kb_E, (const double *)D, cre, cim, mask);
        } else if (out_t == 0) {
            k_kb_scatter<double, float><<<grid, 256, 0, s>>>(
                (double *)out, 2 * ldp, ncols, H.scatter_items[c], n, H.gather_items, H.kb_idx,
                H.kb_p32, H.kb_E, (const float *)D, cre, cim, mask);
        } else {
            k_kb_scatter<float, float><<<grid, 256, 0, s>>>(
                (float *)out, 2 * ldp, ncols, H.scatter_items[c], n, H.gather_items, H.kb_idx,
                H.kb_p32, H.kb_E, (const float *)D, cre, cim, mask);
        }
        RSG_CHECK_HIP(hipGetLastError());
    }
    return RSG_OK;
}

int launch_kb_gather_batch(const KbSys *sys, const int4 *items, int32_t nitems, hipStream_t s) {
    if (nitems == 0) return RSG_OK;
    k_kb_gather_batch<<<(unsigned)nitems, GW * 64, 0, s>>>(sys, items);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

int launch_kb_gather_sum_batch(const KbSys *sys, const int2 *items, int32_t nitems, hipStream_t s) {
    if (nitems == 0) return RSG_OK;
    k_kb_gather_sum_batch<<<(unsigned)nitems, 256, 0, s>>>(sys, items);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

int launch_kb_scatter_batch(const KbSys *sys, const int4 *items, int32_t nitems, double cre, double cim,
                            hipStream_t s) {
    if (nitems == 0) return RSG_OK;
    k_kb_scatter_batch<<<(unsigned)((nitems + 3) / 4), 256, 0, s>>>(sys, items, nitems, cre, cim);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

}  // namespace rsg
