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
// Data layout: an orbital batch is orbital-major, [nst][ldp] complex:
// orbital n holds its values at n*ldp + i for compact point i (z-major, y,
// x), so every orbital is one contiguous field and every grid row of it is
// contiguous.  Mapping onto CDNA4:
//   - one workgroup owns a TX x TY tile of (x, y) columns of one orbital and
//     marches along z over the tile's z-extent (or a chunk of it);
//   - a thread owns one column and keeps its complex value on the planes
//     z-4..z+4 in registers (z taps), plus the planes in flight;
//   - the current plane, with a 4-point x/y halo, is staged in LDS for the
//     x and y taps (two plane buffers used in turn, so one barrier per plane
//     suffices); the halo comes from the neighbouring tiles through L2;
//   - x runs fastest over the threads, so a wave's loads are runs of TX
//     consecutive 16-byte values;
//   - loads of later planes are issued before the current plane is computed
//     (software pipeline, depth PD);
//   - workgroup ids are remapped so that each XCD (own L2) receives a
//     contiguous range of the launch order.
// A tile per workgroup covers many more points than a point-major layout
// with the orbitals of a point side by side would allow in the same
// registers, so far fewer halo values are read per output.
//
// The kernels come in two sets that differ only in the store policy of the
// stage output (NTS: non-temporal stores for outputs much larger than the
// caches); each set is instantiated in a source file of its own.
#pragma once

#include "rsg_internal.h"
#include "stencil_common.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace rsg {
namespace sk {

// Halo assignment of a TX x TY tile (fixed for the whole march): halo value
// j is a y-halo point for j < 8 TX (4 rows above, 4 below, x fastest) and an
// x-halo point otherwise (4 left and 4 right of each tile row).
template <int TX, int TY, int HPT>
struct Halo {
    int l[HPT], x[HPT], y[HPT];
    bool ok[HPT];
    __device__ __forceinline__ Halo(int t, int4 it) {
        constexpr int NT = TX * TY, NHP = 8 * TX + 8 * TY, LX = TX + 8;
#pragma unroll
        for (int k = 0; k < HPT; ++k) {
            const int j = t + k * NT;
            int lxl, lyl;
            if (j < 8 * TX) {
                const int yh = j / TX;
                lxl = j % TX + 4;
                lyl = yh < 4 ? yh : TY + yh;
            } else {
                const int q = j - 8 * TX;
                const int cc = q % 8;
                lyl = q / 8 + 4;
                lxl = cc < 4 ? cc : TX + cc;
            }
            ok[k] = j < NHP;
            if (!ok[k]) lxl = lyl = 0;
            l[k] = lyl * LX + lxl;
            x[k] = it.x * TX + lxl - 4;
            y[k] = it.y * TY + lyl - 4;
        }
    }
};

// The per-point epilogue shared by both marches: H value from the Laplacian
// taps, then the stage combination (times the absorber mask m_c when MASK),
// stored at idx (dropped when idx = -1; zero at the dead slot -idx - 2 when
// idx <= -2).  PAIR (a first-type FP64 stage of the discrete adjoint): b_c
// holds the pair operand u at the point, and pacc gathers conj(in) x_axis u
// (zero wherever the point is outside the box, since both loads read zero
// there).
template <bool NTS, class Tc, class Tout, int MODE, bool FIRST, bool MASK, bool CS, bool PAIR = false>
__device__ __forceinline__ void finish(const KParams &a, typename CT<Tc>::c2 q0, Tc lr, Tc li, Tc v_c,
                                       Tc vi_c, double2 b_c, double m_c, double E, int x, int y, int z,
                                       int idx, __amdgpu_buffer_rsrc_t rout, double2 &pacc) {
    Tc vloc = v_c;
    if constexpr (PAIR || (!std::is_same<Tc, double>::value && FIRST)) {
        // a branch here: in the FP32 first-type stages a select costs
        // registers at the 4-wave occupancy limit, and the pair stages (which
        // always have a field axis) measured the same either way
        if (a.axis >= 0) {
            const int cc = a.axis == 0 ? x : (a.axis == 1 ? y : z);
            const double xc = a.h * ((double)cc - a.off_axis);
            vloc += (Tc)(E * xc);
            if constexpr (PAIR) {
                pacc.x += xc * ((double)q0.x * b_c.x + (double)q0.y * b_c.y);
                pacc.y += xc * ((double)q0.x * b_c.y - (double)q0.y * b_c.x);
            }
        }
    } else {
        // the field term as a select: a branch in the march's step costs
        // more than the few operations it would skip
        const int cc = a.axis == 0 ? x : (a.axis == 1 ? y : z);
        const double xc = a.h * ((double)cc - a.off_axis);
        const Tc vf = vloc + (Tc)(E * xc);
        vloc = a.axis >= 0 ? vf : vloc;
    }
    const Tc kin_h2 = (Tc)a.kin_h2;
    Tc hr, hi;
    if constexpr (CS) {
        // complex kinetic prefactor and complex local potential
        const Tc ki = (Tc)a.kin_h2_im;
        hr = kin_h2 * lr - ki * li + vloc * q0.x - vi_c * q0.y;
        hi = kin_h2 * li + ki * lr + vloc * q0.y + vi_c * q0.x;
    } else {
        hr = kin_h2 * lr + vloc * q0.x;
        hi = kin_h2 * li + vloc * q0.y;
    }
    const bool dead = idx < -1;
    const unsigned o = boff<Tout>(dead ? -idx - 2 : idx);
    if (MODE == 0) {
        store_c<NTS>(rout, o, (Tout *)nullptr, dead ? 0.0 : (double)hr, dead ? 0.0 : (double)hi);
    } else {
        const double2 bb = FIRST ? make_double2((double)q0.x, (double)q0.y) : b_c;
        double r = bb.x + (a.cre * (double)hr - a.cim * (double)hi);
        double i = bb.y + (a.cre * (double)hi + a.cim * (double)hr);
        if (MASK) {
            r *= m_c;
            i *= m_c;
        }
        store_c<NTS>(rout, o, (Tout *)nullptr, dead ? 0.0 : r, dead ? 0.0 : i);
    }
}

// Software-pipelined march, depth D = 1..2, over the item's planes zs, zs +
// dir, ... (dir = +1 upward, -1 downward; the stencil is symmetric in z).
// At step k (output plane z = zs + dir k) a thread
//   - issues the row-table reads for the loads of step k+1,
//   - issues the data loads of plane k+4+D (own column), of the halo of plane
//     k+HA and of V and base at plane k+D, from row entries read one step
//     earlier,
//   - computes plane k from data that arrived during earlier steps.
// HA = 4+D when each thread carries one halo value (the halo of a plane is
// then loaded in the same step as the plane's own columns, by this and by
// the neighbouring workgroups, while the lines are in L2), else HA = D.
// All rings are indexed by compile-time constants after unrolling the step
// loop by a common period, so no register is moved while its load is in
// flight.  FIRST: base == in, whose value at the point is the centre tap.
template <bool NTS, int TX, int TY, int D, class Tin, class Tc, class Tout, int MODE, bool FIRST, bool MASK, bool CS,
          bool PAIR>
__device__ __forceinline__ void march_ring(const KParams &a, const int4 it, const int n,
                                           typename CT<Tc>::c2 *tile, double2 &pacc) {
    using C2 = typename CT<Tc>::c2;
    // selects instead of branches in the row lookups: the row index always,
    // the slot in the row except in the FP32 stage that reads complex128
    // (there that select costs registers at the 4-wave occupancy limit)
    constexpr bool SEL = std::is_same<Tc, double>::value || std::is_same<Tin, float2>::value;
    constexpr int NT = TX * TY, LX = TX + 8;
    constexpr int HPT = (8 * TX + 8 * TY + NT - 1) / NT;
    static_assert(D >= 1 && D <= 2, "pipeline depth 1..2");
    constexpr int Q = D == 1 ? 10 : 12;        // own-column ring, >= 9 + D
    constexpr int HA = HPT == 1 ? 4 + D : D;   // planes ahead at which the halo is loaded
    constexpr int HQ = HA;                     // halo ring slots
    constexpr int VD = D + 1;                  // V / base ring slots
    constexpr int P = clcm(clcm(clcm(clcm(Q, D), VD), 2), HQ);
    constexpr int PLANE = (TY + 8) * LX;       // one plane buffer; tile holds two
    const int t = threadIdx.x, lx = t % TX, ly = t / TX;
    const int x = it.x * TX + lx, y = it.y * TY + ly;
    const int64_t np = a.np;
    const auto rin = rsrc(static_cast<const Tin *>(a.in) + (int64_t)n * a.ldp, np * (int64_t)sizeof(Tin));
    // the base operand (later stages), or the pair operand of an adjoint stage
    const auto rbase = rsrc(static_cast<const double2 *>(PAIR ? a.pair_y : a.base) + (int64_t)n * a.ldp, np * 16);
    const auto rout = rsrc(static_cast<Tout *>(a.out) + (int64_t)n * a.ldp, np * (int64_t)sizeof(Tout));
    const auto rv = rsrc(a.V, np * (int64_t)sizeof(Tc));
    const auto rm = rsrc(MASK ? a.mask : a.V, MASK ? np * 8 : 0);
    const auto rvi = rsrc(CS ? a.Vim : a.V, CS && a.Vim ? np * 8 : 0);
    const Halo<TX, TY, HPT> hl(t, it);

    auto fetch = [&](int idx, bool ok) -> C2 { return load_c<Tc, Tin>(rin, ok ? boff<Tin>(idx) : OOB); };
    auto fetch_v = [&](int idx) -> Tc { return BL<Tc>::ld(rv, boff<Tc>(idx)); };
    auto fetch_b = [&](int idx) -> double2 {
        if (MODE != 1 || (FIRST && !PAIR)) return make_double2(0.0, 0.0);
        return BL<double2>::ld(rbase, boff<double2>(idx));
    };
    auto fetch_m = [&](int idx) -> double { return MASK ? BL<double>::ld(rm, boff<double>(idx)) : 1.0; };
    auto fetch_vi = [&](int idx) -> Tc { return CS ? (Tc)BL<double>::ld(rvi, boff<double>(idx)) : (Tc)0; };

    const int zs = it.z, dir = it.w > it.z ? 1 : -1;
    const int nk = (it.w - it.z) * dir;  // planes to compute
    // prologue: planes k = -4 .. 3+D into ring slots 0 .. Q-2 (slot of plane
    // k is k + 4), halo of planes 0 .. HA-1, V/base of planes 0 .. D-1, rows
    // for step 0.  Every row entry the prologue needs is requested before
    // any is used, so that they arrive in one round trip (taking them one
    // at a time chained a dozen L2 round trips ahead of the first plane);
    // except in the FP32 stage that reads complex128, where holding them
    // all costs registers at the 4-wave occupancy limit.
    constexpr bool HOIST = !(std::is_same<Tc, float>::value && std::is_same<Tin, double2>::value);
    int2 rw[Q - 1];
    int2 rwh[HQ][HPT];
    if constexpr (HOIST) {
#pragma unroll
        for (int j = 0; j < Q - 1; ++j) rw[j] = row_of<true>(a, y, zs + dir * (j - 4));
#pragma unroll
        for (int d = 0; d < HQ; ++d)
#pragma unroll
            for (int k = 0; k < HPT; ++k) rwh[d][k] = row_of<true>(a, hl.y[k], zs + dir * d);
    }
    // step k reads row slot k % 2 and fills the other one
    int2 rfr[2], rhl[2][HPT];
    rfr[0] = row_of<true>(a, y, zs + dir * (4 + D));
#pragma unroll
    for (int k = 0; k < HPT; ++k) rhl[0][k] = row_of<true>(a, hl.y[k], zs + dir * HA);
    rfr[1] = make_int2(0, 0);
#pragma unroll
    for (int k = 0; k < HPT; ++k) rhl[1][k] = make_int2(0, 0);
    C2 cv[Q];
    int oid[Q];
#pragma unroll
    for (int j = 0; j < Q - 1; ++j) {
        int2 r;
        if constexpr (HOIST)
            r = rw[j];
        else
            r = row_of<true>(a, y, zs + dir * (j - 4));
        oid[j] = slot_in_row<SEL>(r, x, a.align);
        cv[j] = fetch(oid[j], true);
    }
    cv[Q - 1] = C2{(Tc)0, (Tc)0};
    oid[Q - 1] = -1;
    C2 hal[HQ][HPT];
#pragma unroll
    for (int d = 0; d < HQ; ++d)
#pragma unroll
        for (int k = 0; k < HPT; ++k) {
            int2 r;
            if constexpr (HOIST)
                r = rwh[d][k];
            else
                r = row_of<true>(a, hl.y[k], zs + dir * d);
            hal[d][k] = fetch(idx_in_row(r, hl.x[k]), hl.ok[k] && d < nk);
        }
    Tc vr[VD], vir[VD];
    double2 br[VD];
    double mr[VD];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        vr[d] = fetch_v(oid[4 + d]);
        vir[d] = fetch_vi(oid[4 + d]);
        br[d] = fetch_b(oid[4 + d]);
        mr[d] = fetch_m(oid[4 + d]);
    }
    vr[D] = (Tc)0;
    vir[D] = (Tc)0;
    br[D] = make_double2(0.0, 0.0);
    mr[D] = 0.0;

    const double E = a.field_dev ? *a.field_dev : a.field;
    const int own = (ly + 4) * LX + lx + 4;

    for (int kb = 0; kb < nk; kb += P) {
#pragma unroll
        for (int s = 0; s < P; ++s) {
            const int k = kb + s;
            if (k >= nk) break;
            const int z = zs + dir * k;
            const int sh = s % HQ, sr = s % 2, srp = (s + 1) % 2;
            const int shl = (s + HA) % HQ;              // halo slot of plane k + HA
            const int sv = s % VD, svn = (s + D) % VD;  // V/base: read slot, load slot
            // ring slot of plane k + m
#define SLOT(m) ((s + (m) + 4 + Q) % Q)
            C2 *const pl = tile + (s % 2) * PLANE;  // plane buffer of this step
            pl[own] = cv[SLOT(0)];
#pragma unroll
            for (int j = 0; j < HPT; ++j)
                if (hl.ok[j]) pl[hl.l[j]] = hal[sh][j];
            const int idx_c = oid[SLOT(0)];
            const Tc v_c = vr[sv];
            const Tc vi_c = vir[sv];
            const double2 b_c = br[sv];
            const double m_c = mr[sv];
            __syncthreads();
            {
                // row entries for the next step first, then the loads that use
                // the entries read last step
                rfr[srp] = row_of<true>(a, y, z + dir * (5 + D));
#pragma unroll
                for (int j = 0; j < HPT; ++j) rhl[srp][j] = row_of<true>(a, hl.y[j], z + dir * (1 + HA));
                int idf;
                if constexpr (SEL) {
                    const int sl = slot_in_row<true>(rfr[sr], x, a.align);
                    idf = (k + 4 + D < nk + 4) ? sl : -1;
                } else {
                    idf = (k + 4 + D < nk + 4) ? slot_in_row<false>(rfr[sr], x, a.align) : -1;
                }
                oid[SLOT(4 + D)] = idf;
                cv[SLOT(4 + D)] = fetch(idf, true);
                const bool hlive = k + HA < nk;
#pragma unroll
                for (int j = 0; j < HPT; ++j)
                    hal[shl][j] = fetch(idx_in_row(rhl[sr][j], hl.x[j]), hl.ok[j] && hlive);
                const int idv = k + D < nk ? oid[SLOT(D)] : -1;
                vr[svn] = fetch_v(idv);
                vir[svn] = fetch_vi(idv);
                br[svn] = fetch_b(idv);
                mr[svn] = fetch_m(idv);
            }
            const C2 q0 = cv[SLOT(0)];
            Tc lr, li;
            {
                const C2 xm1 = pl[own - 1], xp1 = pl[own + 1], xm2 = pl[own - 2], xp2 = pl[own + 2];
                const C2 xm3 = pl[own - 3], xp3 = pl[own + 3], xm4 = pl[own - 4], xp4 = pl[own + 4];
                const C2 ym1 = pl[own - LX], yp1 = pl[own + LX], ym2 = pl[own - 2 * LX], yp2 = pl[own + 2 * LX];
                const C2 ym3 = pl[own - 3 * LX], yp3 = pl[own + 3 * LX], ym4 = pl[own - 4 * LX], yp4 = pl[own + 4 * LX];
                const C2 zm1 = cv[SLOT(-1)], zp1 = cv[SLOT(1)], zm2 = cv[SLOT(-2)], zp2 = cv[SLOT(2)];
                const C2 zm3 = cv[SLOT(-3)], zp3 = cv[SLOT(3)], zm4 = cv[SLOT(-4)], zp4 = cv[SLOT(4)];
                lr = (Tc)3 * FD<Tc>::c0 * q0.x + FD<Tc>::c1 * ((xm1.x + xp1.x) + (ym1.x + yp1.x) + (zm1.x + zp1.x)) +
                     FD<Tc>::c2 * ((xm2.x + xp2.x) + (ym2.x + yp2.x) + (zm2.x + zp2.x)) +
                     FD<Tc>::c3 * ((xm3.x + xp3.x) + (ym3.x + yp3.x) + (zm3.x + zp3.x)) +
                     FD<Tc>::c4 * ((xm4.x + xp4.x) + (ym4.x + yp4.x) + (zm4.x + zp4.x));
                li = (Tc)3 * FD<Tc>::c0 * q0.y + FD<Tc>::c1 * ((xm1.y + xp1.y) + (ym1.y + yp1.y) + (zm1.y + zp1.y)) +
                     FD<Tc>::c2 * ((xm2.y + xp2.y) + (ym2.y + yp2.y) + (zm2.y + zp2.y)) +
                     FD<Tc>::c3 * ((xm3.y + xp3.y) + (ym3.y + yp3.y) + (zm3.y + zp3.y)) +
                     FD<Tc>::c4 * ((xm4.y + xp4.y) + (ym4.y + yp4.y) + (zm4.y + zp4.y));
            }
#undef SLOT
            finish<NTS, Tc, Tout, MODE, FIRST, MASK, CS, PAIR>(a, q0, lr, li, v_c, vi_c, b_c, m_c, E, x, y, z, idx_c, rout,
                                                       pacc);
            // no barrier here: the next step writes the other plane buffer,
            // and every wave has finished reading it once all have passed
            // this step's barrier
        }
    }
}

// Lean march (depth 1, few registers): the own-column queue q[9] rotates in
// registers and every load of plane k+1 (own column k+5, halo, V, base) is
// issued one step ahead; a step starts by waiting for the previous step's
// loads.  Planes run zs, zs + dir, ... as in the pipelined march.
template <bool NTS, int TX, int TY, class Tin, class Tc, class Tout, int MODE, bool FIRST, bool MASK, bool CS,
          bool PAIR>
__device__ __forceinline__ void march_lean(const KParams &a, const int4 it, const int n,
                                           typename CT<Tc>::c2 *tile, double2 &pacc) {
    using C2 = typename CT<Tc>::c2;
    // selects instead of branches in the row lookups: the row index always,
    // the slot in the row in the FP64 kernels (in the FP32 ones that select
    // costs registers at the 4-wave occupancy limit)
    constexpr bool SEL = std::is_same<Tc, double>::value;
    constexpr int NT = TX * TY, LX = TX + 8;
    constexpr int HPT = (8 * TX + 8 * TY + NT - 1) / NT;
    constexpr int PLANE = (TY + 8) * LX;  // one plane buffer; tile holds two
    const int t = threadIdx.x, lx = t % TX, ly = t / TX;
    const int x = it.x * TX + lx, y = it.y * TY + ly;
    const int64_t np = a.np;
    const auto rin = rsrc(static_cast<const Tin *>(a.in) + (int64_t)n * a.ldp, np * (int64_t)sizeof(Tin));
    // the base operand (later stages), or the pair operand of an adjoint stage
    const auto rbase = rsrc(static_cast<const double2 *>(PAIR ? a.pair_y : a.base) + (int64_t)n * a.ldp, np * 16);
    const auto rout = rsrc(static_cast<Tout *>(a.out) + (int64_t)n * a.ldp, np * (int64_t)sizeof(Tout));
    const auto rv = rsrc(a.V, np * (int64_t)sizeof(Tc));
    const auto rm = rsrc(MASK ? a.mask : a.V, MASK ? np * 8 : 0);
    const auto rvi = rsrc(CS ? a.Vim : a.V, CS && a.Vim ? np * 8 : 0);
    const Halo<TX, TY, HPT> hl(t, it);

    auto fetch = [&](int idx, bool ok) -> C2 { return load_c<Tc, Tin>(rin, ok ? boff<Tin>(idx) : OOB); };
    auto fetch_v = [&](int idx) -> Tc { return BL<Tc>::ld(rv, boff<Tc>(idx)); };
    auto fetch_b = [&](int idx) -> double2 {
        if (MODE != 1 || (FIRST && !PAIR)) return make_double2(0.0, 0.0);
        return BL<double2>::ld(rbase, boff<double2>(idx));
    };
    auto fetch_m = [&](int idx) -> double { return MASK ? BL<double>::ld(rm, boff<double>(idx)) : 1.0; };
    auto fetch_vi = [&](int idx) -> Tc { return CS ? (Tc)BL<double>::ld(rvi, boff<double>(idx)) : (Tc)0; };

    const int zs = it.z, dir = it.w > it.z ? 1 : -1;
    const int nk = (it.w - it.z) * dir;
    // every row entry of the prologue is requested before any is used (one
    // round trip, not one per entry)
    int2 rq[9];  // planes zs - 4 .. zs + 4
#pragma unroll
    for (int j = 0; j < 9; ++j) rq[j] = row_of<true>(a, y, zs + dir * (j - 4));
    int2 rh0[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) rh0[j] = row_of<true>(a, hl.y[j], zs);
    int2 rf = row_of<true>(a, y, zs + dir * 5);  // rows for the loads of the first step
    int2 ro = rq[5];                             // plane zs + 1
    int2 rh[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) rh[j] = row_of<true>(a, hl.y[j], zs + dir);
    C2 q[9];
#pragma unroll
    for (int j = 0; j < 8; ++j) q[j] = fetch(idx_in_row(rq[j], x), true);
    int idx_c = slot_in_row<SEL>(rq[4], x, a.align);
    C2 nxt = fetch(idx_in_row(rq[8], x), true);
    C2 hv[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) hv[j] = fetch(idx_in_row(rh0[j], hl.x[j]), hl.ok[j]);
    Tc v_c = fetch_v(idx_c);
    Tc vi_c = fetch_vi(idx_c);
    double2 b_c = fetch_b(idx_c);
    double m_c = fetch_m(idx_c);

    const double E = a.field_dev ? *a.field_dev : a.field;
    const int own = (ly + 4) * LX + lx + 4;

    for (int k = 0; k < nk; ++k) {
        const int z = zs + dir * k;
        C2 *const pl = tile + (k & 1) * PLANE;  // plane buffer of this step
        q[8] = nxt;
        pl[own] = q[4];
#pragma unroll
        for (int j = 0; j < HPT; ++j)
            if (hl.ok[j]) pl[hl.l[j]] = hv[j];
        __syncthreads();
        // row entries for the next step, then this step's loads (plane k+1)
        const int2 rf_n = row_of<true>(a, y, z + dir * 6), ro_n = row_of<true>(a, y, z + dir * 2);
        int2 rh_n[HPT];
#pragma unroll
        for (int j = 0; j < HPT; ++j) rh_n[j] = row_of<true>(a, hl.y[j], z + dir * 2);
        const bool live = k + 1 < nk;
        nxt = fetch(live ? idx_in_row(rf, x) : -1, true);
#pragma unroll
        for (int j = 0; j < HPT; ++j) hv[j] = fetch(idx_in_row(rh[j], hl.x[j]), hl.ok[j] && live);
        const int idx_n = live ? slot_in_row<SEL>(ro, x, a.align) : -1;
        const Tc v_n = fetch_v(idx_n);
        const Tc vi_n = fetch_vi(idx_n);
        const double2 b_n = fetch_b(idx_n);
        const double m_n = fetch_m(idx_n);
        rf = rf_n;
        ro = ro_n;
#pragma unroll
        for (int j = 0; j < HPT; ++j) rh[j] = rh_n[j];

        const C2 q0 = q[4];
        Tc lr, li;
        {
            const C2 xm1 = pl[own - 1], xp1 = pl[own + 1], xm2 = pl[own - 2], xp2 = pl[own + 2];
            const C2 xm3 = pl[own - 3], xp3 = pl[own + 3], xm4 = pl[own - 4], xp4 = pl[own + 4];
            const C2 ym1 = pl[own - LX], yp1 = pl[own + LX], ym2 = pl[own - 2 * LX], yp2 = pl[own + 2 * LX];
            const C2 ym3 = pl[own - 3 * LX], yp3 = pl[own + 3 * LX], ym4 = pl[own - 4 * LX], yp4 = pl[own + 4 * LX];
            lr = (Tc)3 * FD<Tc>::c0 * q0.x + FD<Tc>::c1 * ((xm1.x + xp1.x) + (ym1.x + yp1.x) + (q[3].x + q[5].x)) +
                 FD<Tc>::c2 * ((xm2.x + xp2.x) + (ym2.x + yp2.x) + (q[2].x + q[6].x)) +
                 FD<Tc>::c3 * ((xm3.x + xp3.x) + (ym3.x + yp3.x) + (q[1].x + q[7].x)) +
                 FD<Tc>::c4 * ((xm4.x + xp4.x) + (ym4.x + yp4.x) + (q[0].x + q[8].x));
            li = (Tc)3 * FD<Tc>::c0 * q0.y + FD<Tc>::c1 * ((xm1.y + xp1.y) + (ym1.y + yp1.y) + (q[3].y + q[5].y)) +
                 FD<Tc>::c2 * ((xm2.y + xp2.y) + (ym2.y + yp2.y) + (q[2].y + q[6].y)) +
                 FD<Tc>::c3 * ((xm3.y + xp3.y) + (ym3.y + yp3.y) + (q[1].y + q[7].y)) +
                 FD<Tc>::c4 * ((xm4.y + xp4.y) + (ym4.y + yp4.y) + (q[0].y + q[8].y));
        }
        finish<NTS, Tc, Tout, MODE, FIRST, MASK, CS, PAIR>(a, q0, lr, li, v_c, vi_c, b_c, m_c, E, x, y, z, idx_c, rout,
                                                       pacc);
#pragma unroll
        for (int j = 0; j < 8; ++j) q[j] = q[j + 1];
        idx_c = idx_n;
        v_c = v_n;
        vi_c = vi_n;
        b_c = b_n;
        m_c = m_n;
    }
}

template <bool NTS, int TX, int TY, int D, class Tin, class Tc, class Tout, int MODE, bool FIRST, bool MASK, bool CS,
          bool PAIR = false>
__device__ __forceinline__ void march(const KParams &a, const int4 it, const int n, typename CT<Tc>::c2 *tile,
                                      double2 &pacc) {
    if constexpr (D == 0)
        march_lean<NTS, TX, TY, Tin, Tc, Tout, MODE, FIRST, MASK, CS, PAIR>(a, it, n, tile, pacc);
    else
        march_ring<NTS, TX, TY, D, Tin, Tc, Tout, MODE, FIRST, MASK, CS, PAIR>(a, it, n, tile, pacc);
}

// Sum of v over the workgroup (xor shuffles within each wave, then the wave
// totals in wave order through LDS); thread 0 gets the result.  The caller's
// LDS buffer must be free: a barrier precedes its reuse.
template <int NT>
__device__ __forceinline__ double2 wg_sum(double2 v, double2 *lds) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        v.x += __shfl_xor(v.x, off);
        v.y += __shfl_xor(v.y, off);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double2 s = make_double2(0.0, 0.0);
    if (threadIdx.x == 0)
        for (int w = 0; w < (NT + 63) / 64; ++w) {
            s.x += lds[w].x;
            s.y += lds[w].y;
        }
    return s;
}

template <bool NTS, int TX, int TY, int D, class Tin, class Tc, class Tout, int MODE, bool FIRST, bool MASK = false,
          bool CS = false, bool PAIR = false>
__global__ void __launch_bounds__(TX * TY) k_stencil(KParams a) {
    __shared__ typename CT<Tc>::c2 tile[2 * (TY + 8) * (TX + 8)];  // two plane buffers
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    int n, item;
    block_item(a, blk, &n, &item);
    // uniform by construction; saying so keeps the buffer resources in
    // scalar registers (no per-lane loop around each buffer instruction)
    n = __builtin_amdgcn_readfirstlane(n);
    item = __builtin_amdgcn_readfirstlane(item);
    double2 pacc = make_double2(0.0, 0.0);
    march<NTS, TX, TY, D, Tin, Tc, Tout, MODE, FIRST, MASK, CS, PAIR>(a, a.items[item], n, tile, pacc);
    if constexpr (PAIR) {
        // this workgroup's part of the pair sum, at its place in the launch
        // order (a fixed position, so the final sum has a fixed order)
        const double2 s = wg_sum<TX * TY>(pacc, reinterpret_cast<double2 *>(tile));
        if (threadIdx.x == 0) reinterpret_cast<double2 *>(a.pair_out)[blk] = s;
    }
}

// Persistent form over many independent systems (FP64).  The item list
// {tile, system, orbital} is cut into kBatchQueues contiguous segments of
// about equal work, one per XCD: a workgroup takes the next item of its own
// XCD's segment (workgroup b runs on XCD b mod 8) from that segment's
// counter as soon as it is free, so the items in flight on one XCD are
// neighbours in the list (neighbouring tiles of one system and orbital,
// which then share halo lines in that XCD's L2) however long each march is.
// A workgroup whose segment is used up takes items from the following
// segments in turn.  Each system's parameters come from sysp[system].
// ctr[q] counts the items taken from segment q, ctr[kBatchQueues] the
// workgroups done; the last workgroup out sets them all back to zero for
// the next launch (every workgroup has found every segment used up before
// it counts itself done, so no item is taken after the reset).
template <bool NTS, int TX, int TY, int D, bool FIRST>
__global__ void __launch_bounds__(TX * TY) k_stencil_batch(const KParams *__restrict__ sysp,
                                                           const BatchItem *__restrict__ items,
                                                           const int32_t *__restrict__ seg, double cre,
                                                           double cim, int32_t *ctr) {
    __shared__ double2 tile[2 * (TY + 8) * (TX + 8)];  // two plane buffers
    __shared__ int32_t next;
    const int home = blockIdx.x % kBatchQueues;
    for (int j = 0; j < kBatchQueues; ++j) {
        const int q = (home + j) % kBatchQueues;
        const int32_t s0 = seg[q], s1 = seg[q + 1];
        for (;;) {
            if (threadIdx.x == 0) next = s0 + atomicAdd(&ctr[q], 1);
            __syncthreads();
            const int w = __builtin_amdgcn_readfirstlane(next);
            __syncthreads();  // every thread has read next before it is written again
            if (w >= s1) break;
            const BatchItem bi = items[w];
            KParams a = sysp[__builtin_amdgcn_readfirstlane(bi.sys)];
            a.cre = cre;
            a.cim = cim;
            double2 unused = make_double2(0.0, 0.0);
            march<NTS, TX, TY, D, double2, double, double2, 1, FIRST, false, false>(
                a, bi.tile, __builtin_amdgcn_readfirstlane(bi.ob), tile, unused);
            __syncthreads();  // the next item reuses the plane buffer
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();  // this workgroup's last takes precede its count below
        if (atomicAdd(&ctr[kBatchQueues], 1) == (int)gridDim.x - 1) {
            for (int q = 0; q <= kBatchQueues; ++q) atomicExch(&ctr[q], 0);
        }
    }
}

// Complex-scaled Hamiltonians use the depth-1 pipelined march; other tile
// shapes are mapped to these (see launch_stencil).
template <bool NTS, int TX, int TY, int D>
int launch_fp64_cs(const StageArgs &a, const KParams &p, int nb, hipStream_t s) {
    constexpr int NT = TX * TY;
    if (a.in_t != 0 || a.out_t != 0 || a.mask || a.pair_y) return RSG_EUNSUPPORTED;
    if (a.mode == 0)
        k_stencil<NTS, TX, TY, D, double2, double, double2, 0, false, false, true><<<nb, NT, 0, s>>>(p);
    else if (a.first)
        k_stencil<NTS, TX, TY, D, double2, double, double2, 1, true, false, true><<<nb, NT, 0, s>>>(p);
    else
        k_stencil<NTS, TX, TY, D, double2, double, double2, 1, false, false, true><<<nb, NT, 0, s>>>(p);
    return RSG_OK;
}

template <bool NTS, int TX, int TY, int D>
int launch_fp64(const StageArgs &a, const KParams &p, int nb, hipStream_t s) {
    constexpr int NT = TX * TY;
    if (a.in_t != 0 || a.out_t != 0) return RSG_EUNSUPPORTED;
    if (a.pair_y && !(a.mode == 1 && a.first && !a.mask)) return RSG_EUNSUPPORTED;
    if (a.mode == 0)
        k_stencil<NTS, TX, TY, D, double2, double, double2, 0, false><<<nb, NT, 0, s>>>(p);
    else if (a.pair_y)
        k_stencil<NTS, TX, TY, D, double2, double, double2, 1, true, false, false, true><<<nb, NT, 0, s>>>(p);
    else if (a.first)
        k_stencil<NTS, TX, TY, D, double2, double, double2, 1, true><<<nb, NT, 0, s>>>(p);
    else if (a.mask)
        k_stencil<NTS, TX, TY, D, double2, double, double2, 1, false, true><<<nb, NT, 0, s>>>(p);
    else
        k_stencil<NTS, TX, TY, D, double2, double, double2, 1, false><<<nb, NT, 0, s>>>(p);
    return RSG_OK;
}

// Mixed path: FP32 arithmetic; the first stage reads complex128 psi and
// writes complex64, the middle stages complex64 to complex64 (each its own
// base), the last complex64 to complex128 with the complex128 base psi.
template <bool NTS, int TX, int TY, int D>
int launch_fp32(const StageArgs &a, const KParams &p, int nb, hipStream_t s) {
    constexpr int NT = TX * TY;
    if (a.mode != 1 || a.pair_y) return RSG_EUNSUPPORTED;
    if (a.in_t == 0 && a.out_t == 1 && a.first)
        k_stencil<NTS, TX, TY, D, double2, float, float2, 1, true><<<nb, NT, 0, s>>>(p);
    else if (a.in_t == 1 && a.out_t == 1 && a.first)
        k_stencil<NTS, TX, TY, D, float2, float, float2, 1, true><<<nb, NT, 0, s>>>(p);
    else if (a.in_t == 1 && a.out_t == 0 && !a.first && a.mask)
        k_stencil<NTS, TX, TY, D, float2, float, double2, 1, false, true><<<nb, NT, 0, s>>>(p);
    else if (a.in_t == 1 && a.out_t == 0 && !a.first)
        k_stencil<NTS, TX, TY, D, float2, float, double2, 1, false><<<nb, NT, 0, s>>>(p);
    else
        return RSG_EUNSUPPORTED;
    return RSG_OK;
}

// grid < 0: return the number of resident workgroups of this kernel on the
// device (occupancy query, not allowed during graph capture); grid > 0:
// launch with that many persistent workgroups.
template <bool NTS, int TX, int TY, int D, bool FIRST>
int launch_batch_inst(const KParams *sysp, const BatchItem *items, const int32_t *seg, int32_t nitems, double cre,
                      double cim, int32_t *ctr, int grid, hipStream_t s) {
    constexpr int NT = TX * TY;
    auto kern = k_stencil_batch<NTS, TX, TY, D, FIRST>;
    if (grid < 0) {
        int per_cu = 0, dev = 0;
        hipDeviceProp_t prop;
        RSG_CHECK_HIP(hipGetDevice(&dev));
        RSG_CHECK_HIP(hipGetDeviceProperties(&prop, dev));
        RSG_CHECK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, 0));
        return std::max(1, per_cu) * prop.multiProcessorCount;
    }
    kern<<<(int)std::min<int64_t>(nitems, grid), NT, 0, s>>>(sysp, items, seg, cre, cim, ctr);
    return RSG_OK;
}

template <bool NTS, int TX, int TY, int D>
int launch_batch_shape(bool first, const KParams *sysp, const BatchItem *items, const int32_t *seg, int32_t nitems,
                       double cre, double cim, int32_t *ctr, int grid, hipStream_t s) {
    if (first) return launch_batch_inst<NTS, TX, TY, D, true>(sysp, items, seg, nitems, cre, cim, ctr, grid, s);
    return launch_batch_inst<NTS, TX, TY, D, false>(sysp, items, seg, nitems, cre, cim, ctr, grid, s);
}

}  // namespace sk

// Tile shapes compiled into the library, {TX, TY, depth}: depth 1..2 is the
// pipelined march, depth 0 the lean one.  (Deeper pipelines and 1024-thread
// tiles are not compiled: their rings spill past the register limit.)
#define RSG_FP64_SHAPES(X) \
    X(8, 8, 1) X(8, 8, 2) X(16, 8, 1) X(16, 8, 2) X(32, 8, 1) X(32, 8, 2) X(16, 16, 1) \
    X(16, 16, 2) X(32, 16, 1) X(32, 16, 2) X(64, 8, 1) X(64, 8, 2) X(32, 16, 0)
#define RSG_FP32_SHAPES(X) X(16, 8, 1) X(32, 8, 1) X(32, 8, 2) X(32, 16, 1) X(32, 16, 2) X(64, 8, 2)
#define RSG_CS_SHAPES(X) X(8, 8, 1) X(16, 8, 1) X(16, 16, 1) X(32, 16, 1)

// One stencil stage over nb workgroups with the compiled kernel for the
// tile shape and the stage's types (RSG_EUNSUPPORTED if there is none).
template <bool NTS>
int stencil_dispatch(const StageArgs &a, const KParams &p, const TileShape &shape, bool cs, int nb, hipStream_t s) {
    int rc = RSG_EUNSUPPORTED;
    bool found = false;
#define RSG_TRY(X_, Y_, D_, FN)                                         \
    if (!found && shape.TX == X_ && shape.TY == Y_ && shape.PD == D_) { \
        found = true;                                                   \
        rc = sk::FN<NTS, X_, Y_, D_>(a, p, nb, s);                      \
    }
#define RSG_TRY64(X_, Y_, D_) RSG_TRY(X_, Y_, D_, launch_fp64)
#define RSG_TRY32(X_, Y_, D_) RSG_TRY(X_, Y_, D_, launch_fp32)
#define RSG_TRYCS(X_, Y_, D_) RSG_TRY(X_, Y_, D_, launch_fp64_cs)
    if (shape.B == 1) {
        if (cs) {
            RSG_CS_SHAPES(RSG_TRYCS)
        } else if (a.compute == 0) {
            RSG_FP64_SHAPES(RSG_TRY64)
        } else {
            RSG_FP32_SHAPES(RSG_TRY32)
        }
    }
#undef RSG_TRY64
#undef RSG_TRY32
#undef RSG_TRYCS
#undef RSG_TRY
    return rc;
}

// The persistent batched kernel for the tile shape: grid < 0 returns its
// resident workgroups on the device, grid > 0 launches it with that many
// (RSG_EUNSUPPORTED if the shape is not compiled).
template <bool NTS>
int batch_dispatch(const TileShape &shape, bool first, const KParams *sysp, const BatchItem *items,
                   const int32_t *seg, int32_t nitems, double cre, double cim, int32_t *ctr, int grid, hipStream_t s) {
    int rc = RSG_EUNSUPPORTED;
    bool found = false;
#define RSG_TRY_B(X_, Y_, D_)                                                                             \
    if (!found && shape.TX == X_ && shape.TY == Y_ && shape.PD == D_) {                                   \
        found = true;                                                                                     \
        rc = sk::launch_batch_shape<NTS, X_, Y_, D_>(first, sysp, items, seg, nitems, cre, cim, ctr, grid, s); \
    }
    if (shape.B == 1) { RSG_FP64_SHAPES(RSG_TRY_B) }
#undef RSG_TRY_B
    return rc;
}

// instantiated in stencil_inst.hip (false) and stencil_inst_nt.hip (true)
#define RSG_STENCIL_INST(EXT, NTS_)                                                                           \
    EXT template int stencil_dispatch<NTS_>(const StageArgs &, const KParams &, const TileShape &, bool, int,  \
                                             hipStream_t);                                                    \
    EXT template int batch_dispatch<NTS_>(const TileShape &, bool, const KParams *, const BatchItem *,         \
                                          const int32_t *, int32_t, double, double, int32_t *, int, hipStream_t);
RSG_STENCIL_INST(extern, false)
RSG_STENCIL_INST(extern, true)

}  // namespace rsg
