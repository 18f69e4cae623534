// Two Taylor factors in one z-march: out = (1 + cb L)(1 + ca L) in, with
// L = kin Lap_h + V + E x_axis the local part of H (FP64).  A product-form
// step runs as two such passes instead of four single-factor stages, so
// every point and orbital is read and written once per two applications
// of H instead of once per application.  The projector terms are added
// afterwards by a correction on the projector supports (projector.hip), so
// this kernel is purely local.
//
// Mapping onto CDNA4 (one workgroup = one TX x TY tile of one orbital,
// marching along z):
//   - the first factor runs 4 planes ahead of the second: at step k (output
//     plane z) the first factor computes y1 = (1 + ca L) in at plane z1 =
//     z + 4 on the tile's own columns and on its 4-wide halo band, so that
//     the second factor finds every tap of y1 on chip;
//   - each thread owns one tile column and one band column (8 TX + 8 TY
//     band columns, fewer than TX TY threads): their input planes z .. z+9
//     ride in register rings, and the input plane z1 with an 8-wide halo
//     (own, band, and the outer band and corners that only the band
//     columns' x/y taps need) is staged in LDS buffer A;
//   - y1 of the own column rides in a register ring (planes z-5 .. z+4);
//     y1 of the band columns is parked in a ring of five LDS planes B until
//     the second factor reaches its plane four steps later, and so is V of
//     the own column (read once per pass, used by both factors);
//   - y1 vanishes outside the box (the first factor's result is masked);
//     loads outside the box read zero through the buffer bounds, as in the
//     single-factor march;
//   - all rings are indexed by compile-time constants after unrolling the
//     step loop by 10 (every ring length divides it), so no register moves
//     while its load is in flight.
#include "rsg_internal.h"
#include "stencil_common.h"

namespace rsg {

namespace {

// Column sets of a TX x TY tile, tile-local coordinates (0,0) = first own
// column:
//   band  j < 8 TX:  y-band rows -4..-1 and TY..TY+3 over x 0..TX-1;
//         j < 8 TX + 8 TY: x-band columns -4..-1 and TX..TX+3 over y 0..TY-1;
//   outer j < 8 TX:  rows -8..-5 and TY+4..TY+7 over x 0..TX-1;
//         j < 8 TX + 8 TY: columns -8..-5 and TX+4..TX+7 over y 0..TY-1;
//         j < 8 TX + 8 TY + 64: the four 4 x 4 corners next to the tile.
template <int TX, int TY>
__device__ __forceinline__ void band_col(int j, int *lx, int *ly) {
    if (j < 8 * TX) {
        const int r = j / TX;
        *lx = j % TX;
        *ly = r < 4 ? r - 4 : TY + r - 4;
    } else {
        const int q = j - 8 * TX, c = q % 8;
        *ly = q / 8;
        *lx = c < 4 ? c - 4 : TX + c - 4;
    }
}
template <int TX, int TY>
__device__ __forceinline__ void outer_col(int j, int *lx, int *ly) {
    if (j < 8 * TX) {
        const int r = j / TX;
        *lx = j % TX;
        *ly = r < 4 ? r - 8 : TY + r;
    } else if (j < 8 * TX + 8 * TY) {
        const int q = j - 8 * TX, c = q % 8;
        *ly = q / 8;
        *lx = c < 4 ? c - 8 : TX + c;
    } else {
        const int q = j - 8 * TX - 8 * TY, b = q / 16, w = q % 16;
        *lx = (b & 1) ? TX + w % 4 : w % 4 - 4;
        *ly = (b & 2) ? TY + w / 4 : w / 4 - 4;
    }
}

// Laplacian taps of the value at LDS position p (row length LX) with the z
// neighbours zm[m-1] / zp[m-1] = the value at z -/+ m: returns sum c_|m| of
// the 25-point star (without 1/h^2).
template <int LX>
__device__ __forceinline__ double2 lap25(const double2 *pl, int p, double2 q0, const double2 zm[4],
                                         const double2 zp[4]) {
    using F = FD<double>;
    const double2 xm1 = pl[p - 1], xp1 = pl[p + 1], xm2 = pl[p - 2], xp2 = pl[p + 2];
    const double2 xm3 = pl[p - 3], xp3 = pl[p + 3], xm4 = pl[p - 4], xp4 = pl[p + 4];
    const double2 ym1 = pl[p - LX], yp1 = pl[p + LX], ym2 = pl[p - 2 * LX], yp2 = pl[p + 2 * LX];
    const double2 ym3 = pl[p - 3 * LX], yp3 = pl[p + 3 * LX], ym4 = pl[p - 4 * LX], yp4 = pl[p + 4 * LX];
    double2 r;
    r.x = 3.0 * F::c0 * q0.x + F::c1 * ((xm1.x + xp1.x) + (ym1.x + yp1.x) + (zm[0].x + zp[0].x)) +
          F::c2 * ((xm2.x + xp2.x) + (ym2.x + yp2.x) + (zm[1].x + zp[1].x)) +
          F::c3 * ((xm3.x + xp3.x) + (ym3.x + yp3.x) + (zm[2].x + zp[2].x)) +
          F::c4 * ((xm4.x + xp4.x) + (ym4.x + yp4.x) + (zm[3].x + zp[3].x));
    r.y = 3.0 * F::c0 * q0.y + F::c1 * ((xm1.y + xp1.y) + (ym1.y + yp1.y) + (zm[0].y + zp[0].y)) +
          F::c2 * ((xm2.y + xp2.y) + (ym2.y + yp2.y) + (zm[1].y + zp[1].y)) +
          F::c3 * ((xm3.y + xp3.y) + (ym3.y + yp3.y) + (zm[2].y + zp[2].y)) +
          F::c4 * ((xm4.y + xp4.y) + (ym4.y + yp4.y) + (zm[3].y + zp[3].y));
    return r;
}

// q + c (kin_h2 lap + v q) for complex c = (cr, ci).
__device__ __forceinline__ double2 factor(double2 q, double2 lap, double v, double kin_h2, double cr, double ci) {
    const double hr = kin_h2 * lap.x + v * q.x, hi = kin_h2 * lap.y + v * q.y;
    return make_double2(q.x + (cr * hr - ci * hi), q.y + (cr * hi + ci * hr));
}

template <int TX, int TY>
__global__ void __launch_bounds__(TX * TY) k_fused2(KParams a, double car, double cai, double cbr, double cbi) {
    constexpr int NT = TX * TY;
    constexpr int HC = 8 * TX + 8 * TY;       // band columns
    constexpr int OC = 8 * TX + 8 * TY + 64;  // outer columns and corners
    static_assert(HC <= NT && OC <= NT, "one band and one outer column per thread");
    constexpr int LA = TX + 16, PA = (TY + 16) * LA;  // LDS plane A (input, 8-wide halo)
    constexpr int LB = TX + 8, PB = (TY + 8) * LB;    // LDS plane B (y1, 4-wide halo)
    constexpr int P = 10;                             // unroll period: every ring length divides it
    __shared__ double2 lds[2 * PA + 5 * PB];
    __shared__ double vring[5 * NT];  // V of the own column at plane z1, kept for the second factor
    double2 *const A0 = lds;
    double2 *const B0 = lds + 2 * PA;

    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    int n, item;
    block_item(a, blk, &n, &item);
    n = __builtin_amdgcn_readfirstlane(n);
    item = __builtin_amdgcn_readfirstlane(item);
    const int4 it = a.items[item];

    const int t = threadIdx.x, lx = t % TX, ly = t / TX;
    const int x = it.x * TX + lx, y = it.y * TY + ly;
    int blx, bly, olx, oly;
    band_col<TX, TY>(t < HC ? t : 0, &blx, &bly);
    outer_col<TX, TY>(t < OC ? t : 0, &olx, &oly);
    const bool bok = t < HC, ook = t < OC;
    const int bx = it.x * TX + blx, by = it.y * TY + bly;
    const int ox = it.x * TX + olx, oy = it.y * TY + oly;
    const int ownA = (ly + 8) * LA + lx + 8, bandA = (bly + 8) * LA + blx + 8, outA = (oly + 8) * LA + olx + 8;
    const int ownB = (ly + 4) * LB + lx + 4, bandB = (bly + 4) * LB + blx + 4;

    const int64_t np = a.np;
    const auto rin = rsrc(static_cast<const double2 *>(a.in) + (int64_t)n * a.ldp, np * 16);
    const auto rout = rsrc(static_cast<double2 *>(a.out) + (int64_t)n * a.ldp, np * 16);
    const auto rv = rsrc(a.V, np * 8);
    auto fetch = [&](int idx) -> double2 { return BL<double2>::ld(rin, boff<double2>(idx)); };
    auto fetch_v = [&](int idx) -> double { return BL<double>::ld(rv, boff<double>(idx)); };

    const int zs = it.z, dir = it.w > it.z ? 1 : -1;
    const int nk = (it.w - it.z) * dir;
    const double E = a.field_dev ? *a.field_dev : a.field;
    const double kin_h2 = a.kin_h2;
    const int ax = a.axis;
    auto xcoord = [&](int cx, int cy, int cz) -> double {
        const int cc = ax == 0 ? cx : (ax == 1 ? cy : cz);
        return a.h * ((double)cc - a.off[ax < 0 ? 0 : ax]);
    };

    // step j = k + 8 >= 0 (k = -8 .. nk-1): output plane z = zs + dir k,
    // first-factor plane z1 = z + 4 dir.  Input ring slot of plane zs + dir m
    // (m >= -8) is (m + 8) % 10, so plane z + d sits in slot (j + d) % 10.
    double2 cv[P], cb[P];  // input at the own / band column
    // their compact indices: the own column's is its slot (a dead slot of a
    // row-aligned grid encoded <= -2, which loads read as zero and the
    // store fills with zero), the band column's -1 outside the box
    int oid[P], bid[P];
#pragma unroll
    for (int d = 0; d < 9; ++d) {
        const int z = zs + dir * (d - 8);
        oid[d] = slot_in_row(row_of(a, y, z), x, a.align);
        bid[d] = bok ? idx_in_row(row_of(a, by, z), bx) : -1;
        cv[d] = fetch(oid[d]);
        cb[d] = fetch(bid[d]);
    }
    oid[9] = bid[9] = -1;
    cv[9] = cb[9] = make_double2(0.0, 0.0);
    // outer column input at plane z1, two slots by step parity
    double2 co[2];
    co[0] = fetch(ook ? idx_in_row(row_of(a, oy, zs - 4 * dir), ox) : -1);
    co[1] = make_double2(0.0, 0.0);
    // V at the own / band column for plane z1 of step j (slot j % 2)
    double vo[2], vb[2];
    vo[0] = fetch_v(oid[4]);
    vb[0] = fetch_v(bid[4]);
    vo[1] = vb[1] = 0.0;
    // y1 at the own column, plane zs + dir m in slot (m + 8) % 10
    double2 y1[P];
#pragma unroll
    for (int d = 0; d < P; ++d) y1[d] = make_double2(0.0, 0.0);
    // row entries for the loads of the next step: input plane z + 9 (own,
    // band), outer plane z1 + 1
    int2 ro = row_of(a, y, zs + dir), rb = row_of(a, by, zs + dir), rx = row_of(a, oy, zs - 3 * dir);

    const int nsteps = nk + 8;
    for (int jb = 0; jb < nsteps; jb += P) {
#pragma unroll
        for (int s = 0; s < P; ++s) {
            const int j = jb + s;
            if (j >= nsteps) break;
            const int k = j - 8;
            const int z = zs + dir * k, z1 = z + 4 * dir;
            double2 *const Aq = A0 + (s % 2) * PA;
            double2 *const Bq = B0 + (s % 5) * PB;         // y1 at plane z
            double2 *const Bn = B0 + ((s + 4) % 5) * PB;   // y1 at plane z1 (band part)
            double *const Vq = vring + (s % 5) * NT, *const Vn = vring + ((s + 4) % 5) * NT;
#define IS(d) ((s + (d)) % P)
            // stage the input plane z1 in A and the own y1 of plane z in B
            Aq[ownA] = cv[IS(4)];
            if (bok) Aq[bandA] = cb[IS(4)];
            if (ook) Aq[outA] = co[s % 2];
            if (k >= 0) Bq[ownB] = y1[IS(0)];
            __syncthreads();
            {
                // loads for the next step: input plane z + 9, outer plane
                // z1 + 1, V at plane z1 + 1; row entries for the step after
                const int2 ron = row_of(a, y, z + 10 * dir), rbn = row_of(a, by, z + 10 * dir);
                const int2 rxn = row_of(a, oy, z1 + 2 * dir);
                const bool live = j + 1 < nsteps;
                const int io = live ? slot_in_row(ro, x, a.align) : -1;
                const int ib = live && bok ? idx_in_row(rb, bx) : -1;
                oid[IS(9)] = io;
                bid[IS(9)] = ib;
                cv[IS(9)] = fetch(io);
                cb[IS(9)] = fetch(ib);
                co[(s + 1) % 2] = fetch(live && ook ? idx_in_row(rx, ox) : -1);
                vo[(s + 1) % 2] = fetch_v(live ? oid[IS(5)] : -1);
                vb[(s + 1) % 2] = fetch_v(live ? bid[IS(5)] : -1);
                ro = ron;
                rb = rbn;
                rx = rxn;
            }
            // first factor at plane z1: own column and band column
            {
                const double2 zm[4] = {cv[IS(3)], cv[IS(2)], cv[IS(1)], cv[IS(0)]};
                const double2 zp[4] = {cv[IS(5)], cv[IS(6)], cv[IS(7)], cv[IS(8)]};
                const double2 q = cv[IS(4)];
                const double2 l = lap25<LA>(Aq, ownA, q, zm, zp);
                Vn[t] = vo[s % 2];
                const double v = vo[s % 2] + (ax >= 0 ? E * xcoord(x, y, z1) : 0.0);
                const double2 r = factor(q, l, v, kin_h2, car, cai);
                y1[IS(4)] = oid[IS(4)] >= 0 ? r : make_double2(0.0, 0.0);
            }
            if (bok) {
                const double2 zm[4] = {cb[IS(3)], cb[IS(2)], cb[IS(1)], cb[IS(0)]};
                const double2 zp[4] = {cb[IS(5)], cb[IS(6)], cb[IS(7)], cb[IS(8)]};
                const double2 q = cb[IS(4)];
                const double2 l = lap25<LA>(Aq, bandA, q, zm, zp);
                const double v = vb[s % 2] + (ax >= 0 ? E * xcoord(bx, by, z1) : 0.0);
                const double2 r = factor(q, l, v, kin_h2, car, cai);
                Bn[bandB] = bid[IS(4)] >= 0 ? r : make_double2(0.0, 0.0);
            }
            // second factor at plane z (own column), from y1
            if (k >= 0) {
                const int own_store = oid[IS(0)];
                const double2 zm[4] = {y1[IS(-1 + P)], y1[IS(-2 + P)], y1[IS(-3 + P)], y1[IS(-4 + P)]};
                const double2 zp[4] = {y1[IS(1)], y1[IS(2)], y1[IS(3)], y1[IS(4)]};
                const double2 q = y1[IS(0)];
                const double2 l = lap25<LB>(Bq, ownB, q, zm, zp);
                // V at plane z was loaded for the first factor four steps ago
                const double v = Vq[t] + (ax >= 0 ? E * xcoord(x, y, z) : 0.0);
                const double2 r = factor(q, l, v, kin_h2, cbr, cbi);
                const bool dead = own_store < -1;
                BL<double2>::st(rout, boff<double2>(dead ? -own_store - 2 : own_store),
                                dead ? make_double2(0.0, 0.0) : r);
            }
#undef IS
        }
    }
}

template <int TX, int TY>
int launch_fused_shape(const KParams &p, int nb, double2 ca, double2 cb, hipStream_t s) {
    k_fused2<TX, TY><<<nb, TX * TY, 0, s>>>(p, ca.x, ca.y, cb.x, cb.y);
    return RSG_OK;
}

}  // namespace

// Fused tile shapes: one band and one outer column per thread.
#define RSG_FUSED_SHAPES(X) X(32, 16)

std::vector<TileShape> fused_candidates() {
    std::vector<TileShape> v;
#define RSG_ADDF(X_, Y_)            \
    {                               \
        TileShape sh{1, X_, Y_, 0}; \
        sh.PD = 1;                  \
        sh.FU = 1;                  \
        v.push_back(sh);            \
    }
    RSG_FUSED_SHAPES(RSG_ADDF)
#undef RSG_ADDF
    return v;
}

int launch_fused(const Ham &H, const FusedArgs &f, const TileShape &tile, hipStream_t s) {
    const Grid &g = *H.g;
    if (H.complex_scaled()) {
        set_error("fused stencil: complex-scaled Hamiltonians use single-factor stages");
        return RSG_EUNSUPPORTED;
    }
    int err = RSG_OK;
    TileShape shape = tile;
    if (shape.ZC <= 0) shape.ZC = g.n[2];
    const TilePlan *plan = const_cast<Grid &>(g).plan(shape, s, &err);
    if (!plan) return err;
    if (plan->nitems == 0 || f.nst == 0) return RSG_OK;
    if (g.np >= (int64_t)(0x80000000u / 16)) {
        set_error("fused stencil: grids of 2^27 points or more are not supported");
        return RSG_EUNSUPPORTED;
    }
    StageArgs a;
    a.in = f.in;
    a.base = f.in;
    a.out = f.out;
    a.mode = 1;
    a.first = true;
    a.nst = f.nst;
    a.ldp = f.ldp;
    a.field = f.field;
    a.field_dev = f.field_dev;
    const KParams p = make_params(H, a, shape, plan);
    const int64_t nb64 = (int64_t)plan->nitems * f.nst;
    if (nb64 > INT32_MAX) {
        set_error("fused stencil launch too large");
        return RSG_EUNSUPPORTED;
    }
    const double2 ca = make_double2(f.ca.real(), f.ca.imag()), cb = make_double2(f.cb.real(), f.cb.imag());
    int rc = RSG_EUNSUPPORTED;
    bool found = false;
    timing_before(s);
#define RSG_TRYF(X_, Y_)                                                   \
    if (!found && shape.TX == X_ && shape.TY == Y_) {                      \
        found = true;                                                      \
        rc = launch_fused_shape<X_, Y_>(p, (int)nb64, ca, cb, s);          \
    }
    RSG_FUSED_SHAPES(RSG_TRYF)
#undef RSG_TRYF
    timing_after(s);
    if (rc == RSG_EUNSUPPORTED) {
        set_error("fused stencil: unsupported tile %dx%d", shape.TX, shape.TY);
        return rc;
    }
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

}  // namespace rsg
