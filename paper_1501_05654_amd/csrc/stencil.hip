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

struct KParams {
    const void *in;
    const void *base;
    void *out;
    const int4 *items;
    const int2 *rows;
    const void *V;
    const double *field_dev;
    int64_t nst, ld;
    double kin_h2;
    double field;
    double h;
    double off[3];
    double cre, cim;
    int32_t nob;
    int32_t ny, nz;
    int32_t axis;
};

// Workgroup b of nb runs on XCD b % 8; give each XCD a contiguous range.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, local = b >> 3;
    return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + local;
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

template <int B, int TX, int TY, class Tin, class Tc, int MODE, class Tout>
__global__ void __launch_bounds__(B * TX * TY) k_stencil(KParams a) {
    using C2 = typename CT<Tc>::c2;
    constexpr int NT = B * TX * TY;
    constexpr int LX = TX + 8, LY = TY + 8;
    constexpr int NHP = 8 * TX + 8 * TY;  // halo points of one plane
    constexpr int NH = NHP * B;
    constexpr int HPT = (NH + NT - 1) / NT;
    __shared__ C2 tile[LY * LX * B];

    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int item = blk / a.nob, ob = blk - item * a.nob;
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

template <int B, int TX, int TY, class Tin, class Tc, int MODE, class Tout>
int launch_one(const KParams &p, int nblocks, hipStream_t s) {
    k_stencil<B, TX, TY, Tin, Tc, MODE, Tout><<<nblocks, B * TX * TY, 0, s>>>(p);
    return RSG_OK;
}

// Type combinations used by the library: FP64 throughout, and the mixed
// path (FP32 Hamiltonian on complex64 or complex128 input, FP64 base).
template <int B, int TX, int TY>
int dispatch_types(const StageArgs &a, const KParams &p, int nblocks, hipStream_t s) {
    if (a.compute == 0) {
        if (a.in_t != 0 || a.out_t != 0) return RSG_EUNSUPPORTED;
        return a.mode == 0 ? launch_one<B, TX, TY, double2, double, 0, double2>(p, nblocks, s)
                           : launch_one<B, TX, TY, double2, double, 1, double2>(p, nblocks, s);
    }
    if (a.mode != 1) return RSG_EUNSUPPORTED;
    if (a.in_t == 0 && a.out_t == 1) return launch_one<B, TX, TY, double2, float, 1, float2>(p, nblocks, s);
    if (a.in_t == 1 && a.out_t == 1) return launch_one<B, TX, TY, float2, float, 1, float2>(p, nblocks, s);
    if (a.in_t == 1 && a.out_t == 0) return launch_one<B, TX, TY, float2, float, 1, double2>(p, nblocks, s);
    return RSG_EUNSUPPORTED;
}

}  // namespace

// FP64 uses 512-thread tiles (about 150 VGPRs, no spills); the FP32 path
// fits 1024-thread tiles in registers.
TileShape default_shape(const Grid &g, int64_t nst, int compute) {
    TileShape sh;
    if (nst <= 1) sh = {1, 16, 16, 0};
    else if (nst <= 2) sh = {2, 16, 16, 0};
    else if (nst <= 4) sh = compute == 0 ? TileShape{4, 16, 8, 0} : TileShape{4, 16, 16, 0};
    else sh = compute == 0 ? TileShape{8, 8, 8, 0} : TileShape{8, 16, 8, 0};
    sh.ZC = g.n[2];
    return sh;
}

int launch_stencil(const Ham &H, const StageArgs &a, const TileShape &shape, hipStream_t s) {
    const Grid &g = *H.g;
    int err = RSG_OK;
    TileShape key = shape;
    if (key.ZC <= 0) key.ZC = g.n[2];
    const TilePlan *plan = const_cast<Grid &>(g).plan(key, s, &err);
    if (!plan) return err;
    if (plan->nitems == 0 || a.nst == 0) return RSG_OK;
    KParams p;
    p.in = a.in;
    p.base = a.base;
    p.out = a.out;
    p.items = plan->items;
    p.rows = g.rows;
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
    p.ny = g.n[1];
    p.nz = g.n[2];
    p.axis = H.axis;
    const int64_t nb64 = (int64_t)plan->nitems * p.nob;
    if (nb64 > INT32_MAX) {
        set_error("stencil launch too large");
        return RSG_EUNSUPPORTED;
    }
    const int nb = (int)nb64;
    timing_before(s);
    int rc = RSG_EUNSUPPORTED;
#define RSG_SHAPE(B_, X_, Y_) \
    if (shape.B == B_ && shape.TX == X_ && shape.TY == Y_) rc = dispatch_types<B_, X_, Y_>(a, p, nb, s);
    RSG_SHAPE(1, 16, 16)
    else RSG_SHAPE(2, 16, 16)
    else RSG_SHAPE(4, 16, 16)
    else RSG_SHAPE(4, 16, 8)
    else RSG_SHAPE(8, 16, 8)
    else RSG_SHAPE(8, 8, 8)
#undef RSG_SHAPE
    timing_after(s);
    if (rc == RSG_EUNSUPPORTED) {
        set_error("stencil: unsupported tile shape %dx%dx%d / type combination", shape.B, shape.TX,
                  shape.TY);
        return rc;
    }
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

}  // namespace rsg
