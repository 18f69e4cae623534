// Kinetic + local-potential part of H applied to an orbital batch, with the
// Taylor-stage epilogue fused in.
//
//   (H psi)(r) = kin/h^2 sum_axes sum_{m=-4..4} c_|m| psi(r + m h e_axis)
//              + (V(r) + E x_axis(r)) psi(r)
//
// c_0..c_4 = -205/72, 8/5, -1/5, 8/315, -1/560 (8th-order centred second
// derivative); orbitals vanish outside the box.  High-order finite
// differences are the discretisation of the section "Introduction"; the
// order is this library's choice.  The separable projectors are added by the
// projector kernels after this one.
//
// Data layout: an orbital batch is [np][ld] complex, orbital index fastest,
// points in compact order (z-major, y, x).  Mapping onto CDNA4:
//   - one workgroup owns a TX x TY tile of (x, y) columns and B orbitals, and
//     marches along z over the tile's z-extent (or a chunk of it);
//   - each thread keeps its own column's 9 planes (z-4..z+4) in registers,
//     so every orbital value is read from memory once per workgroup for the
//     z taps;
//   - the current plane, with a 4-point x/y halo, is staged in LDS for the
//     x and y taps; halo values come from neighbouring tiles through L2;
//   - lanes run over orbitals first, so a wave reads B*16 contiguous bytes
//     per point, and consecutive points of a row are contiguous;
//   - the next plane and the next halo are fetched into registers before the
//     current plane is computed (one plane of prefetch);
//   - workgroup ids are remapped so that each XCD (own L2) receives a
//     contiguous range of tiles.
#include "rsg_internal.h"

#include <algorithm>

namespace rsg {

namespace {

template <class Tc> struct CT;
template <> struct CT<double> { using c2 = double2; };
template <> struct CT<float> { using c2 = float2; };

template <class Tc>
struct FD {
    static constexpr Tc c0 = (Tc)(-205.0 / 72.0);
    static constexpr Tc c1 = (Tc)(8.0 / 5.0);
    static constexpr Tc c2 = (Tc)(-1.0 / 5.0);
    static constexpr Tc c3 = (Tc)(8.0 / 315.0);
    static constexpr Tc c4 = (Tc)(-1.0 / 560.0);
};

// Workgroup b of nb runs on XCD b % 8; give each XCD a contiguous range.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, local = b >> 3;
    return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + local;
}

// Block order.  Batch fastest: the orbital batches of a tile run together,
// so the whole ld-orbital row of each point is read at about the same time
// (DRAM row locality).  Batch slowest: each XCD sweeps a band of tiles of one
// batch, so neighbouring tiles can find each other's halos in L2.
__device__ __forceinline__ void block_item(const KParams &a, int blk, int *ob, int *item) {
    if (a.batch_slowest) {
        *ob = blk / a.nitems;
        *item = blk - *ob * a.nitems;
    } else {
        *item = blk / a.nob;
        *ob = blk - *item * a.nob;
    }
}

__device__ __forceinline__ int64_t point_index(const KParams &a, int x, int y, int z) {
    if (y < 0 || y >= a.ny || z < 0 || z >= a.nz) return -1;
    const int2 r = a.rows[z * a.ny + y];
    const int x0 = r.y & 0xffff, x1 = (r.y >> 16) & 0xffff;
    if (x < x0 || x >= x1) return -1;
    return (int64_t)r.x + x;
}

__device__ __forceinline__ void store_c(double2 *p, double r, double i) { *p = make_double2(r, i); }
__device__ __forceinline__ void store_c(float2 *p, double r, double i) {
    *p = make_float2((float)r, (float)i);
}
__device__ __forceinline__ void store_c(double2 *p, float r, float i) {
    *p = make_double2((double)r, (double)i);
}
__device__ __forceinline__ void store_c(float2 *p, float r, float i) { *p = make_float2(r, i); }

template <class Tin, class Tc>
__device__ __forceinline__ typename CT<Tc>::c2 fetch(const Tin *in, int64_t idx, int64_t ld,
                                                     int64_t s, bool ok) {
    using C2 = typename CT<Tc>::c2;
    if (!ok || idx < 0) return C2{(Tc)0, (Tc)0};
    const Tin v = in[idx * ld + s];
    return C2{(Tc)v.x, (Tc)v.y};
}

// Complex-lane variant (one complex value per lane), used by the mixed
// path: FP32 arithmetic on complex64 or complex128 input.
template <int B, int TX, int TY, class Tin, class Tc, int MODE, class Tout>
__global__ void __launch_bounds__(B * TX * TY) k_stencil_c(KParams a) {
    using C2 = typename CT<Tc>::c2;
    constexpr int NT = B * TX * TY;
    constexpr int LX = TX + 8, LY = TY + 8;
    constexpr int NHP = 8 * TX + 8 * TY;  // halo points of one plane
    constexpr int NH = NHP * B;
    constexpr int HPT = (NH + NT - 1) / NT;
    __shared__ C2 tile[LY * LX * B];

    const int blk = xcd_remap(blockIdx.x, gridDim.x);  // block order: see k_stencil_r
    int ob, item;
    block_item(a, blk, &ob, &item);
    const int4 it = a.items[item];
    const int t = threadIdx.x;
    const int o = t % B, lx = (t / B) % TX, ly = t / (B * TX);
    const int x = it.x * TX + lx, y = it.y * TY + ly;
    const int64_t s = (int64_t)ob * B + o;
    const bool sok = s < a.nst;
    const Tin *in = static_cast<const Tin *>(a.in);

    // Halo assignment (fixed for the whole march): value j = t + k*NT is
    // orbital j % B of halo point j / B.  Points 0..8TX-1 are the y halo rows
    // (x fastest), the rest the x halo columns (4 left, 4 right per row).
    int hl[HPT], hx[HPT], hy[HPT];
    int64_t hs[HPT];
    bool hok[HPT];
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
        const int j = t + k * NT;
        const int oh = j % B, hp = j / B;
        int lxl, lyl;
        if (hp < 8 * TX) {
            const int yh = hp / TX;
            lxl = hp % TX + 4;
            lyl = yh < 4 ? yh : TY + yh;
        } else {
            const int q = hp - 8 * TX;
            const int c = q % 8;
            lyl = q / 8 + 4;
            lxl = c < 4 ? c : TX + c;
        }
        hl[k] = (lyl * LX + lxl) * B + oh;
        hx[k] = it.x * TX + lxl - 4;
        hy[k] = it.y * TY + lyl - 4;
        hs[k] = (int64_t)ob * B + oh;
        hok[k] = j < NH && hs[k] < a.nst;
    }

    const int z0 = it.z, z1 = it.w;
    C2 q[9];
#pragma unroll
    for (int k = 0; k < 8; ++k) q[k] = fetch<Tin, Tc>(in, point_index(a, x, y, z0 - 4 + k), a.ld, s, sok);
    C2 nxt = fetch<Tin, Tc>(in, point_index(a, x, y, z0 + 4), a.ld, s, sok);
    C2 hv[HPT];
#pragma unroll
    for (int k = 0; k < HPT; ++k) hv[k] = fetch<Tin, Tc>(in, point_index(a, hx[k], hy[k], z0), a.ld, hs[k], hok[k]);

    const double E = a.field_dev ? *a.field_dev : a.field;
    const Tc kin_h2 = (Tc)a.kin_h2;
    const Tc *Vp = static_cast<const Tc *>(a.V);
    const int own_l = ((ly + 4) * LX + lx + 4) * B + o;

    for (int z = z0; z < z1; ++z) {
        q[8] = nxt;
        tile[own_l] = q[4];
#pragma unroll
        for (int k = 0; k < HPT; ++k)
            if (t + k * NT < NH) tile[hl[k]] = hv[k];
        __syncthreads();
        if (z + 1 < z1) {
            nxt = fetch<Tin, Tc>(in, point_index(a, x, y, z + 5), a.ld, s, sok);
#pragma unroll
            for (int k = 0; k < HPT; ++k)
                hv[k] = fetch<Tin, Tc>(in, point_index(a, hx[k], hy[k], z + 1), a.ld, hs[k], hok[k]);
        }
        const int64_t idx = point_index(a, x, y, z);
        if (idx >= 0 && sok) {
            const C2 cc = q[4];
            const C2 xm1 = tile[own_l - B], xp1 = tile[own_l + B];
            const C2 xm2 = tile[own_l - 2 * B], xp2 = tile[own_l + 2 * B];
            const C2 xm3 = tile[own_l - 3 * B], xp3 = tile[own_l + 3 * B];
            const C2 xm4 = tile[own_l - 4 * B], xp4 = tile[own_l + 4 * B];
            constexpr int YS = LX * B;
            const C2 ym1 = tile[own_l - YS], yp1 = tile[own_l + YS];
            const C2 ym2 = tile[own_l - 2 * YS], yp2 = tile[own_l + 2 * YS];
            const C2 ym3 = tile[own_l - 3 * YS], yp3 = tile[own_l + 3 * YS];
            const C2 ym4 = tile[own_l - 4 * YS], yp4 = tile[own_l + 4 * YS];
            C2 lap;
            lap.x = (Tc)3 * FD<Tc>::c0 * cc.x +
                    FD<Tc>::c1 * ((xm1.x + xp1.x) + (ym1.x + yp1.x) + (q[3].x + q[5].x)) +
                    FD<Tc>::c2 * ((xm2.x + xp2.x) + (ym2.x + yp2.x) + (q[2].x + q[6].x)) +
                    FD<Tc>::c3 * ((xm3.x + xp3.x) + (ym3.x + yp3.x) + (q[1].x + q[7].x)) +
                    FD<Tc>::c4 * ((xm4.x + xp4.x) + (ym4.x + yp4.x) + (q[0].x + q[8].x));
            lap.y = (Tc)3 * FD<Tc>::c0 * cc.y +
                    FD<Tc>::c1 * ((xm1.y + xp1.y) + (ym1.y + yp1.y) + (q[3].y + q[5].y)) +
                    FD<Tc>::c2 * ((xm2.y + xp2.y) + (ym2.y + yp2.y) + (q[2].y + q[6].y)) +
                    FD<Tc>::c3 * ((xm3.y + xp3.y) + (ym3.y + yp3.y) + (q[1].y + q[7].y)) +
                    FD<Tc>::c4 * ((xm4.y + xp4.y) + (ym4.y + yp4.y) + (q[0].y + q[8].y));
            Tc vloc = Vp ? Vp[idx] : (Tc)0;
            if (a.axis >= 0) {
                const int c = a.axis == 0 ? x : (a.axis == 1 ? y : z);
                vloc += (Tc)(E * (a.h * ((double)c - a.off[a.axis])));
            }
            const Tc hr = kin_h2 * lap.x + vloc * cc.x;
            const Tc hi = kin_h2 * lap.y + vloc * cc.y;
            Tout *out = static_cast<Tout *>(a.out);
            if (MODE == 0) {
                store_c(out + idx * a.ld + s, hr, hi);
            } else {
                const double2 bb = static_cast<const double2 *>(a.base)[idx * a.ld + s];
                const double r = bb.x + (a.cre * (double)hr - a.cim * (double)hi);
                const double i = bb.y + (a.cre * (double)hi + a.cim * (double)hr);
                store_c(out + idx * a.ld + s, r, i);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8; ++k) q[k] = q[k + 1];
    }
}

// Real-lane variant for FP64: lanes run over the 2*nst real columns of the
// interleaved batch (re and im of an orbital in adjacent lanes), so a thread
// carries one double per plane instead of a complex pair; the Horner
// epilogue gets the partner component with one xor-1 lane shuffle.
//
// Software pipeline over z, depth D: at step z (output plane z) a thread
//   - issues the row-table reads for the loads of step z+1,
//   - issues the data loads of plane z+4+D (own column, entering the
//     register queue D steps later), of the halo of plane z+D, and the V and
//     base values of plane z+D, all from row entries read one step earlier,
//   - computes plane z from data that arrived during earlier steps.
// No load is waited on in the step that issues it, and no data load waits on
// a row-table read of the same step.  FIRST: base == in, whose value at the
// point is the centre tap.
// Branch-free row lookup: an out-of-box row reads the empty sentinel entry
// that follows the table.  Loads are never masked after they return (the
// compiler would place the select where the load is issued and wait there);
// a masked-off lane loads from a location that holds the neutral value.
__device__ __forceinline__ int2 row_of(const KParams &a, int y, int z) {
    const bool v = y >= 0 && y < a.ny && z >= 0 && z < a.nz;
    return a.rows[v ? z * a.ny + y : a.ny * a.nz];
}
__device__ __forceinline__ int idx_in_row(int2 r, int x) {
    const int x0 = r.y & 0xffff, x1 = (r.y >> 16) & 0xffff;
    return (x >= x0 && x < x1) ? r.x + x : -1;
}

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }
constexpr int clcm(int a, int b) { return a / cgcd(a, b) * b; }

// One work item of the FP64 kernel: tile it = (tx, ty, z0, z1), orbital
// batch ob, with the shared-memory plane `tile` of the calling workgroup.
template <int RB, int TX, int TY, int MODE, bool FIRST, int D>
__device__ __forceinline__ void march_r(const KParams &a, const int4 it, const int ob, double *tile) {
    constexpr int NT = RB * TX * TY;
    constexpr int LX = TX + 8;
    constexpr int NHP = 8 * TX + 8 * TY;
    constexpr int NH = NHP * RB;
    constexpr int HPT = (NH + NT - 1) / NT;
    constexpr int YS = LX * RB;
    // Register rings, all indexed by compile-time constants after unrolling:
    //   col[Q]  own-column values of planes z-4 .. z+4+D (loads land in place),
    //   oid[Q]  own compact index of the same planes,
    //   hal[D]: halo of planes z .. z+D-1,
    //   vr[D+1], br[D+1]: V and base, loaded into the slot consumed last step
    //     so that a new load never targets a register still being read,
    //   rfr[2], rhl[2]: row entries read one step before the loads using them.
    constexpr int Q = D == 1 ? 10 : 12;  // >= 9 + D, and keeps the unroll period at 10 or 12
    constexpr int VD = D + 1;
    constexpr int P = clcm(clcm(clcm(Q, D), VD), 2);  // unroll period of the z loop
    const int t = threadIdx.x;
    const int c = t % RB, lx = (t / RB) % TX, ly = t / (RB * TX);
    const int x = it.x * TX + lx, y = it.y * TY + ly;
    const int ncols = (int)(2 * a.nst);
    const int col = ob * RB + c;
    const bool cok = col < ncols;
    const int64_t ldr = 2 * a.ld;
    const double *in = static_cast<const double *>(a.in);
    const double *base = static_cast<const double *>(a.base);
    const double *Vp = static_cast<const double *>(a.V);

    int hl[HPT], hx[HPT], hy[HPT], hc[HPT];
    bool hok[HPT];
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
        const int j = t + k * NT;
        const int oh = j % RB, hp = j / RB;
        int lxl, lyl;
        if (hp < 8 * TX) {
            const int yh = hp / TX;
            lxl = hp % TX + 4;
            lyl = yh < 4 ? yh : TY + yh;
        } else {
            const int q = hp - 8 * TX;
            const int cc = q % 8;
            lyl = q / 8 + 4;
            lxl = cc < 4 ? cc : TX + cc;
        }
        hl[k] = (lyl * LX + lxl) * RB + oh;
        hx[k] = it.x * TX + lxl - 4;
        hy[k] = it.y * TY + lyl - 4;
        hc[k] = ob * RB + oh;
        hok[k] = j < NH && hc[k] < ncols;
    }
    // Loads are unconditional: a tap outside the box (or a padding column)
    // reads the zero pad; V and base of an outside point read a valid entry
    // whose value is never stored.
    const double *zp = a.zeros;
    auto fetch = [&](int idx, int cc, bool ok) -> double {
        const double *pa = (ok && idx >= 0) ? in + (int64_t)idx * ldr + cc : zp;
        return *pa;
    };
    auto fetch_v = [&](int idx) -> double { return Vp[idx >= 0 ? idx : 0]; };
    auto fetch_b = [&](int idx) -> double {
        if (MODE != 1 || FIRST) return 0.0;
        const bool v = idx >= 0 && cok;
        return base[(int64_t)(v ? idx : 0) * ldr + (v ? col : 0)];
    };

    const int z0 = it.z, z1 = it.w;
    // prologue: planes z0-4 .. z0+3+D into ring slots 0 .. Q-2 (slot of plane
    // z0 + m is m + 4), halo/V/base of planes z0 .. z0+D-1, rows for step z0
    double cv[Q];
    int oid[Q];
#pragma unroll
    for (int j = 0; j < Q - 1; ++j) {
        oid[j] = idx_in_row(row_of(a, y, z0 - 4 + j), x);
        cv[j] = fetch(oid[j], col, cok);
    }
    cv[Q - 1] = 0.0;
    oid[Q - 1] = -1;
    double hal[D][HPT], vr[VD], br[VD];
#pragma unroll
    for (int d = 0; d < D; ++d) {
#pragma unroll
        for (int k = 0; k < HPT; ++k)
            hal[d][k] = fetch(idx_in_row(row_of(a, hy[k], z0 + d), hx[k]), hc[k], hok[k]);
        vr[d] = fetch_v(oid[4 + d]);
        br[d] = fetch_b(oid[4 + d]);
    }
    vr[D] = 0.0;
    br[D] = 0.0;
    // step z reads row slot (z - z0) % 2 and fills the other one
    int2 rfr[2], rhl[2][HPT];
    rfr[0] = row_of(a, y, z0 + 4 + D);
#pragma unroll
    for (int k = 0; k < HPT; ++k) rhl[0][k] = row_of(a, hy[k], z0 + D);
    rfr[1] = make_int2(0, 0);
#pragma unroll
    for (int k = 0; k < HPT; ++k) rhl[1][k] = make_int2(0, 0);

    const double E = a.field_dev ? *a.field_dev : a.field;
    const double kin_h2 = a.kin_h2;
    const int own = ((ly + 4) * LX + lx + 4) * RB + c;
    double *out = static_cast<double *>(a.out);

    for (int zb = z0; zb < z1; zb += P) {
#pragma unroll
        for (int s = 0; s < P; ++s) {
            const int z = zb + s;
            if (z >= z1) break;
            const int sd = s % D, sr = s % 2, srp = (s + 1) % 2;
            const int sv = s % VD, svn = (s + D) % VD;  // V/base: read slot, load slot
            // ring slot of plane z + m
#define SLOT(m) ((s + (m) + 4 + Q) % Q)
            tile[own] = cv[SLOT(0)];
#pragma unroll
            for (int k = 0; k < HPT; ++k)
                if (t + k * NT < NH) tile[hl[k]] = hal[sd][k];
            const int idx_c = oid[SLOT(0)];
            const double v_c = vr[sv], b_c = br[sv];
            __syncthreads();
            {
                // row entries for the next step first, then the loads that use
                // the entries read last step: own column plane z+4+D, halo and
                // V/base of plane z+D
                rfr[srp] = row_of(a, y, z + 5 + D);
#pragma unroll
                for (int k = 0; k < HPT; ++k) rhl[srp][k] = row_of(a, hy[k], z + 1 + D);
                const int idf = (z + 4 + D < z1 + 4) ? idx_in_row(rfr[sr], x) : -1;
                oid[SLOT(4 + D)] = idf;
                cv[SLOT(4 + D)] = fetch(idf, col, cok);
                const bool live = z + D < z1;
#pragma unroll
                for (int k = 0; k < HPT; ++k)
                    hal[sd][k] = fetch(idx_in_row(rhl[sr][k], hx[k]), hc[k], hok[k] && live);
                const int idv = live ? oid[SLOT(D)] : -1;
                vr[svn] = fetch_v(idv);
                br[svn] = fetch_b(idv);
            }
            const double q0 = cv[SLOT(0)];
            const double lap =
                3.0 * FD<double>::c0 * q0 +
                FD<double>::c1 * ((tile[own - RB] + tile[own + RB]) + (tile[own - YS] + tile[own + YS]) + (cv[SLOT(-1)] + cv[SLOT(1)])) +
                FD<double>::c2 * ((tile[own - 2 * RB] + tile[own + 2 * RB]) + (tile[own - 2 * YS] + tile[own + 2 * YS]) + (cv[SLOT(-2)] + cv[SLOT(2)])) +
                FD<double>::c3 * ((tile[own - 3 * RB] + tile[own + 3 * RB]) + (tile[own - 3 * YS] + tile[own + 3 * YS]) + (cv[SLOT(-3)] + cv[SLOT(3)])) +
                FD<double>::c4 * ((tile[own - 4 * RB] + tile[own + 4 * RB]) + (tile[own - 4 * YS] + tile[own + 4 * YS]) + (cv[SLOT(-4)] + cv[SLOT(4)]));
#undef SLOT
            double vloc = v_c;
            if (a.axis >= 0) {
                const int cc = a.axis == 0 ? x : (a.axis == 1 ? y : z);
                vloc += E * (a.h * ((double)cc - a.off[a.axis]));
            }
            const double hval = kin_h2 * lap + vloc * q0;
            if (MODE == 0) {
                if (idx_c >= 0 && cok) out[(int64_t)idx_c * ldr + col] = hval;
            } else {
                const double hpart = __shfl_xor(hval, 1);  // the other component of this orbital
                const double bb = FIRST ? q0 : b_c;
                // re: b + cre*Hre - cim*Him ; im: b + cre*Him + cim*Hre
                const double r = (c & 1) ? bb + (a.cre * hval + a.cim * hpart)
                                         : bb + (a.cre * hval - a.cim * hpart);
                if (idx_c >= 0 && cok) out[(int64_t)idx_c * ldr + col] = r;
            }
            __syncthreads();
        }
    }
}

// Lean variant (pipeline depth 1): the own-column queue q[9] rotates in
// registers and every load of plane z+1 (own column z+5, halo, V, base) is
// issued one step ahead; a step starts by waiting for the previous step's
// loads.  Few registers, so 1024-thread workgroups with 512-point tiles fit
// without spilling, which cuts the halo per output.
template <int RB, int TX, int TY, int MODE, bool FIRST>
__device__ __forceinline__ void march_s(const KParams &a, const int4 it, const int ob, double *tile) {
    constexpr int NT = RB * TX * TY;
    constexpr int LX = TX + 8;
    constexpr int NHP = 8 * TX + 8 * TY;
    constexpr int NH = NHP * RB;
    constexpr int HPT = (NH + NT - 1) / NT;
    constexpr int YS = LX * RB;
    const int t = threadIdx.x;
    const int c = t % RB, lx = (t / RB) % TX, ly = t / (RB * TX);
    const int x = it.x * TX + lx, y = it.y * TY + ly;
    const int ncols = (int)(2 * a.nst);
    const int col = ob * RB + c;
    const bool cok = col < ncols;
    const int64_t ldr = 2 * a.ld;
    const double *in = static_cast<const double *>(a.in);
    const double *base = static_cast<const double *>(a.base);
    const double *Vp = static_cast<const double *>(a.V);
    const double *zp = a.zeros;

    int hl[HPT], hx[HPT], hy[HPT], hc[HPT];
    bool hok[HPT];
#pragma unroll
    for (int k = 0; k < HPT; ++k) {
        const int j = t + k * NT;
        const int oh = j % RB, hp = j / RB;
        int lxl, lyl;
        if (hp < 8 * TX) {
            const int yh = hp / TX;
            lxl = hp % TX + 4;
            lyl = yh < 4 ? yh : TY + yh;
        } else {
            const int q = hp - 8 * TX;
            const int cc = q % 8;
            lyl = q / 8 + 4;
            lxl = cc < 4 ? cc : TX + cc;
        }
        hl[k] = (lyl * LX + lxl) * RB + oh;
        hx[k] = it.x * TX + lxl - 4;
        hy[k] = it.y * TY + lyl - 4;
        hc[k] = ob * RB + oh;
        hok[k] = j < NH && hc[k] < ncols;
    }
    auto fetch = [&](int idx, int cc, bool ok) -> double {
        const double *pa = (ok && idx >= 0) ? in + (int64_t)idx * ldr + cc : zp;
        return *pa;
    };
    auto fetch_v = [&](int idx) -> double { return Vp[idx >= 0 ? idx : 0]; };
    auto fetch_b = [&](int idx) -> double {
        if (MODE != 1 || FIRST) return 0.0;
        const bool v = idx >= 0 && cok;
        return base[(int64_t)(v ? idx : 0) * ldr + (v ? col : 0)];
    };

    const int z0 = it.z, z1 = it.w;
    double q[9];
#pragma unroll
    for (int k = 0; k < 8; ++k) q[k] = fetch(idx_in_row(row_of(a, y, z0 - 4 + k), x), col, cok);
    int idx_c = idx_in_row(row_of(a, y, z0), x);
    double nxt = fetch(idx_in_row(row_of(a, y, z0 + 4), x), col, cok);
    double hv[HPT];
#pragma unroll
    for (int k = 0; k < HPT; ++k) hv[k] = fetch(idx_in_row(row_of(a, hy[k], z0), hx[k]), hc[k], hok[k]);
    double v_c = fetch_v(idx_c), b_c = fetch_b(idx_c);
    int2 rf = row_of(a, y, z0 + 5);  // rows for the loads of the first step
    int2 ro = row_of(a, y, z0 + 1);
    int2 rh[HPT];
#pragma unroll
    for (int k = 0; k < HPT; ++k) rh[k] = row_of(a, hy[k], z0 + 1);

    const double E = a.field_dev ? *a.field_dev : a.field;
    const double kin_h2 = a.kin_h2;
    const int own = ((ly + 4) * LX + lx + 4) * RB + c;
    double *out = static_cast<double *>(a.out);

    for (int z = z0; z < z1; ++z) {
        q[8] = nxt;
        tile[own] = q[4];
#pragma unroll
        for (int k = 0; k < HPT; ++k)
            if (t + k * NT < NH) tile[hl[k]] = hv[k];
        __syncthreads();
        // row entries for the next step, then this step's loads (plane z+1)
        const int2 rf_n = row_of(a, y, z + 6), ro_n = row_of(a, y, z + 2);
        int2 rh_n[HPT];
#pragma unroll
        for (int k = 0; k < HPT; ++k) rh_n[k] = row_of(a, hy[k], z + 2);
        const bool live = z + 1 < z1;
        nxt = fetch(live ? idx_in_row(rf, x) : -1, col, cok);
#pragma unroll
        for (int k = 0; k < HPT; ++k) hv[k] = fetch(idx_in_row(rh[k], hx[k]), hc[k], hok[k] && live);
        const int idx_n = live ? idx_in_row(ro, x) : -1;
        const double v_n = fetch_v(idx_n), b_n = fetch_b(idx_n);
        rf = rf_n;
        ro = ro_n;
#pragma unroll
        for (int k = 0; k < HPT; ++k) rh[k] = rh_n[k];

        const double lap =
            3.0 * FD<double>::c0 * q[4] +
            FD<double>::c1 * ((tile[own - RB] + tile[own + RB]) + (tile[own - YS] + tile[own + YS]) + (q[3] + q[5])) +
            FD<double>::c2 * ((tile[own - 2 * RB] + tile[own + 2 * RB]) + (tile[own - 2 * YS] + tile[own + 2 * YS]) + (q[2] + q[6])) +
            FD<double>::c3 * ((tile[own - 3 * RB] + tile[own + 3 * RB]) + (tile[own - 3 * YS] + tile[own + 3 * YS]) + (q[1] + q[7])) +
            FD<double>::c4 * ((tile[own - 4 * RB] + tile[own + 4 * RB]) + (tile[own - 4 * YS] + tile[own + 4 * YS]) + (q[0] + q[8]));
        double vloc = v_c;
        if (a.axis >= 0) {
            const int cc = a.axis == 0 ? x : (a.axis == 1 ? y : z);
            vloc += E * (a.h * ((double)cc - a.off[a.axis]));
        }
        const double hval = kin_h2 * lap + vloc * q[4];
        if (MODE == 0) {
            if (idx_c >= 0 && cok) out[(int64_t)idx_c * ldr + col] = hval;
        } else {
            const double hpart = __shfl_xor(hval, 1);  // the other component of this orbital
            const double bb = FIRST ? q[4] : b_c;
            const double r = (c & 1) ? bb + (a.cre * hval + a.cim * hpart)
                                     : bb + (a.cre * hval - a.cim * hpart);
            if (idx_c >= 0 && cok) out[(int64_t)idx_c * ldr + col] = r;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8; ++k) q[k] = q[k + 1];
        idx_c = idx_n;
        v_c = v_n;
        b_c = b_n;
    }
}

template <int RB, int TX, int TY, int MODE, bool FIRST, int D>
__global__ void __launch_bounds__(RB * TX * TY) k_stencil_r(KParams a) {
    __shared__ double tile[(TY + 8) * (TX + 8) * RB];
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    int ob, item;
    block_item(a, blk, &ob, &item);
    if constexpr (D == 0)
        march_s<RB, TX, TY, MODE, FIRST>(a, a.items[item], ob, tile);
    else
        march_r<RB, TX, TY, MODE, FIRST, D>(a, a.items[item], ob, tile);
}

// Persistent form over many independent systems: workgroup g takes items
// g, g + G, g + 2G, ... of the cost-sorted list {system, tx, ty, z0, z1, ob};
// each system's parameters come from sysp[system].
template <int RB, int TX, int TY, int MODE, bool FIRST, int D>
__global__ void __launch_bounds__(RB * TX * TY) k_stencil_batch(const KParams *__restrict__ sysp,
                                                                const BatchItem *__restrict__ items,
                                                                int32_t nitems, double cre, double cim) {
    __shared__ double tile[(TY + 8) * (TX + 8) * RB];
    for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
        const BatchItem bi = items[w];
        KParams a = sysp[bi.sys];
        a.cre = cre;
        a.cim = cim;
        if constexpr (D == 0)
            march_s<RB, TX, TY, MODE, FIRST>(a, bi.tile, bi.ob, tile);
        else
            march_r<RB, TX, TY, MODE, FIRST, D>(a, bi.tile, bi.ob, tile);
        __syncthreads();  // the next item reuses the plane buffer
    }
}

template <int B, int TX, int TY>
int launch_c(const StageArgs &a, const KParams &p, int nb, hipStream_t s) {
    constexpr int NT = B * TX * TY;
    if (a.compute == 0 || a.mode != 1) return RSG_EUNSUPPORTED;
    if (a.in_t == 0 && a.out_t == 1)
        k_stencil_c<B, TX, TY, double2, float, 1, float2><<<nb, NT, 0, s>>>(p);
    else if (a.in_t == 1 && a.out_t == 1)
        k_stencil_c<B, TX, TY, float2, float, 1, float2><<<nb, NT, 0, s>>>(p);
    else if (a.in_t == 1 && a.out_t == 0)
        k_stencil_c<B, TX, TY, float2, float, 1, double2><<<nb, NT, 0, s>>>(p);
    else
        return RSG_EUNSUPPORTED;
    return RSG_OK;
}

template <int RB, int TX, int TY, int D>
int launch_rd(const StageArgs &a, const KParams &p, int nb, hipStream_t s) {
    constexpr int NT = RB * TX * TY;
    if (a.mode == 0)
        k_stencil_r<RB, TX, TY, 0, false, D><<<nb, NT, 0, s>>>(p);
    else if (a.first)
        k_stencil_r<RB, TX, TY, 1, true, D><<<nb, NT, 0, s>>>(p);
    else
        k_stencil_r<RB, TX, TY, 1, false, D><<<nb, NT, 0, s>>>(p);
    return RSG_OK;
}

template <int B, int TX, int TY>
int launch_r(const StageArgs &a, const KParams &p, int nb, hipStream_t s, int D) {
    constexpr int RB = 2 * B;
    if (a.compute != 0 || a.in_t != 0 || a.out_t != 0) return RSG_EUNSUPPORTED;
    if (D == 0) return launch_rd<RB, TX, TY, 0>(a, p, nb, s);
    if (RB * TX * TY > 512) return RSG_EUNSUPPORTED;  // deeper pipelines spill at 1024 threads
    if (D == 1) return launch_rd<RB, TX, TY, 1>(a, p, nb, s);
    if (D == 2) return launch_rd<RB, TX, TY, 2>(a, p, nb, s);
    return launch_rd<RB, TX, TY, 3>(a, p, nb, s);
    return RSG_OK;
}

}  // namespace

// Tile shapes compiled into the library: {orbitals per workgroup B, TX, TY}.
// FP64 kernels have 2B real lanes per point, FP32 kernels B complex lanes.
#define RSG_FP64_SHAPES(X) \
    X(1, 16, 16) X(2, 16, 8) X(2, 8, 8) X(4, 8, 8) X(4, 16, 4) X(4, 8, 4) \
    X(8, 8, 4) X(8, 4, 8) X(8, 4, 4) X(16, 4, 4) \
    X(1, 32, 16) X(2, 16, 16) X(4, 16, 8) X(8, 8, 8) X(16, 8, 4) X(16, 4, 8) X(32, 4, 4)
#define RSG_FP32_SHAPES(X) X(1, 16, 16) X(2, 16, 16) X(4, 16, 16) X(4, 16, 8) X(8, 16, 8) X(8, 8, 8)

std::vector<TileShape> tile_candidates(int compute) {
    std::vector<TileShape> shapes, v;
#define RSG_ADD(B_, X_, Y_) shapes.push_back(TileShape{B_, X_, Y_, 0});
    if (compute == 0) {
        RSG_FP64_SHAPES(RSG_ADD)
    } else {
        RSG_FP32_SHAPES(RSG_ADD)
    }
#undef RSG_ADD
    const int d0 = compute == 0 ? 0 : 1, maxd = compute == 0 ? 3 : 1;
    for (int d = d0; d <= maxd; ++d)
        for (auto sh : shapes) {
            if (compute == 0 && d > 0 && 2 * sh.B * sh.TX * sh.TY > 512) continue;
            sh.PD = d;
            v.push_back(sh);
        }
    return v;
}

TileShape default_shape(const Grid &g, int64_t nst, int compute) {
    TileShape sh;
    if (compute == 0) {
        // measured on MI355X (sphere of 3.05 M points): 8 orbitals per
        // workgroup (one 128-byte line per point), 4 x 8 tiles, depth 3,
        // batch-slowest order; fewer orbitals use the lean variant
        if (nst <= 1) sh = {1, 16, 16, 0, 0};
        else if (nst <= 2) sh = {2, 16, 8, 0, 0};
        else if (nst <= 4) sh = {4, 8, 8, 0, 0};
        else {
            sh = {8, 4, 8, 0, 3};
            sh.BO = 1;
        }
    } else {
        if (nst <= 1) sh = {1, 16, 16, 0};
        else if (nst <= 2) sh = {2, 16, 16, 0};
        else if (nst <= 4) sh = {4, 16, 16, 0};
        else sh = {8, 16, 8, 0};
    }
    sh.ZC = g.n[2];
    return sh;
}

TileShape Ham::tile_for(int64_t nst, int compute) const {
    auto it = tiles.find(std::make_pair(nst, compute));
    if (it != tiles.end()) return it->second;
    return default_shape(*g, nst, compute);
}

KParams make_params(const Ham &H, const StageArgs &a, const TileShape &shape, const TilePlan *plan) {
    const Grid &g = *H.g;
    KParams p;
    p.in = a.in;
    p.base = a.base;
    p.out = a.out;
    p.items = plan->items;
    p.rows = g.rows;
    p.zeros = g.zeros;
    p.V = a.compute == 0 ? (const void *)H.V : (const void *)H.V32;
    p.field_dev = a.field_dev;
    p.nst = a.nst;
    p.ld = a.ld;
    p.kin_h2 = H.kin / (g.h * g.h);
    p.field = a.field;
    p.h = g.h;
    for (int k = 0; k < 3; ++k) p.off[k] = 0.5 * (double)(g.n[k] - 1);
    p.cre = a.cre;
    p.cim = a.cim;
    p.nob = (int32_t)((a.nst + shape.B - 1) / shape.B);
    p.nitems = plan ? plan->nitems : 0;
    p.batch_slowest = shape.BO;
    p.ny = g.n[1];
    p.nz = g.n[2];
    p.axis = H.axis;
    return p;
}

int launch_stencil(const Ham &H, const StageArgs &a, const TileShape &shape, hipStream_t s) {
    const Grid &g = *H.g;
    int err = RSG_OK;
    TileShape key = shape;
    if (key.ZC <= 0) key.ZC = g.n[2];
    const TilePlan *plan = const_cast<Grid &>(g).plan(key, s, &err);
    if (!plan) return err;
    if (plan->nitems == 0 || a.nst == 0) return RSG_OK;
    const KParams p = make_params(H, a, shape, plan);
    const int64_t nb64 = (int64_t)plan->nitems * p.nob;
    if (nb64 > INT32_MAX) {
        set_error("stencil launch too large");
        return RSG_EUNSUPPORTED;
    }
    const int nb = (int)nb64;
    timing_before(s);
    int rc = RSG_EUNSUPPORTED;
    bool found = false;
#define RSG_TRY_R(B_, X_, Y_) \
    if (!found && shape.B == B_ && shape.TX == X_ && shape.TY == Y_) { found = true; rc = launch_r<B_, X_, Y_>(a, p, nb, s, shape.PD); }
#define RSG_TRY_C(B_, X_, Y_) \
    if (!found && shape.B == B_ && shape.TX == X_ && shape.TY == Y_) { found = true; rc = launch_c<B_, X_, Y_>(a, p, nb, s); }
    if (a.compute == 0) { RSG_FP64_SHAPES(RSG_TRY_R) } else { RSG_FP32_SHAPES(RSG_TRY_C) }
#undef RSG_TRY_R
#undef RSG_TRY_C
    timing_after(s);
    if (rc == RSG_EUNSUPPORTED) {
        set_error("stencil: unsupported tile shape %dx%dx%d for this precision", shape.B, shape.TX,
                  shape.TY);
        return rc;
    }
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

namespace {
// grid < 0: return the number of resident workgroups of this kernel on the
// device (occupancy query, not allowed during graph capture); grid > 0:
// launch with that many persistent workgroups.
template <int RB, int TX, int TY, int MODE, bool FIRST, int D>
int launch_batch_inst(const KParams *sysp, const BatchItem *items, int32_t nitems, double cre, double cim,
                      int grid, hipStream_t s) {
    constexpr int NT = RB * TX * TY;
    auto kern = k_stencil_batch<RB, TX, TY, MODE, FIRST, D>;
    if (grid < 0) {
        int per_cu = 0, dev = 0;
        hipDeviceProp_t prop;
        RSG_CHECK_HIP(hipGetDevice(&dev));
        RSG_CHECK_HIP(hipGetDeviceProperties(&prop, dev));
        RSG_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, 0));
        return std::max(1, per_cu) * prop.multiProcessorCount;
    }
    kern<<<(int)std::min<int64_t>(nitems, grid), NT, 0, s>>>(sysp, items, nitems, cre, cim);
    return RSG_OK;
}

template <int B, int TX, int TY>
int launch_batch_shape(int mode, bool first, int D, const KParams *sysp, const BatchItem *items, int32_t nitems,
                       double cre, double cim, int grid, hipStream_t s) {
    constexpr int RB = 2 * B;
#define RSG_BD(DD)                                                                                          \
    if (D == DD) {                                                                                          \
        if (mode == 0) return launch_batch_inst<RB, TX, TY, 0, false, DD>(sysp, items, nitems, cre, cim, grid, s); \
        if (first) return launch_batch_inst<RB, TX, TY, 1, true, DD>(sysp, items, nitems, cre, cim, grid, s);      \
        return launch_batch_inst<RB, TX, TY, 1, false, DD>(sysp, items, nitems, cre, cim, grid, s);               \
    }
    RSG_BD(0)
    if (RB * TX * TY > 512) return RSG_EUNSUPPORTED;
    RSG_BD(1) RSG_BD(2) RSG_BD(3)
#undef RSG_BD
    return RSG_EUNSUPPORTED;
}
}  // namespace

int stencil_batch_grid(const TileShape &shape, bool first) {
    int g = RSG_EUNSUPPORTED;
    bool found = false;
#define RSG_TRY_G(B_, X_, Y_)                                                                          \
    if (!found && shape.B == B_ && shape.TX == X_ && shape.TY == Y_) {                                 \
        found = true;                                                                                  \
        g = launch_batch_shape<B_, X_, Y_>(1, first, shape.PD, nullptr, nullptr, 0, 0.0, 0.0, -1, nullptr); \
    }
    RSG_FP64_SHAPES(RSG_TRY_G)
#undef RSG_TRY_G
    return g;
}

int launch_stencil_batch(const TileShape &shape, int mode, bool first, const KParams *sysp,
                         const BatchItem *items, int32_t nitems, double cre, double cim, int grid,
                         hipStream_t s) {
    if (nitems == 0) return RSG_OK;
    if (grid <= 0) {
        set_error("batched stencil: persistent grid size must be > 0");
        return RSG_EINVAL;
    }
    int rc = RSG_EUNSUPPORTED;
    bool found = false;
    timing_before(s);
#define RSG_TRY_B(B_, X_, Y_)                                                                              \
    if (!found && shape.B == B_ && shape.TX == X_ && shape.TY == Y_) {                                     \
        found = true;                                                                                      \
        rc = launch_batch_shape<B_, X_, Y_>(mode, first, shape.PD, sysp, items, nitems, cre, cim, grid, s); \
    }
    RSG_FP64_SHAPES(RSG_TRY_B)
#undef RSG_TRY_B
    timing_after(s);
    if (rc != RSG_OK) {
        if (rc == RSG_EUNSUPPORTED) set_error("batched stencil: unsupported tile %dx%dx%d", shape.B, shape.TX, shape.TY);
        return rc;
    }
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

}  // namespace rsg
