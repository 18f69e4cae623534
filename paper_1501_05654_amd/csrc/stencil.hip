// Host side of the stencil stage: the tile shapes compiled into the library,
// the default shape for a grid, the kernel parameters of a stage and the
// launch (kernels and their dispatch over tile shapes in stencil_kernels.h).
// A stage whose output is at least kNtStoreBytes runs the kernel set with
// non-temporal output stores: such an output is not read again before it
// has left every cache, and streaming it past L2 leaves L2 to the input
// planes and halo lines that neighbouring tiles still read.
#include "stencil_kernels.h"

namespace rsg {

std::vector<TileShape> tile_candidates(int compute) {
    std::vector<TileShape> v;
#define RSG_ADD(X_, Y_, D_)                \
    {                                      \
        TileShape sh{1, X_, Y_, 0};        \
        sh.PD = D_;                        \
        v.push_back(sh);                   \
    }
    if (compute == 0) {
        RSG_FP64_SHAPES(RSG_ADD)
    } else {
        RSG_FP32_SHAPES(RSG_ADD)
    }
#undef RSG_ADD
    return v;
}

// Measured on MI355X (sphere of 3.05 M points, 64 orbitals): 32 x 16 tiles,
// depth 2, orbital-slowest order.  Smaller grids take the largest tile that
// still gives every compute unit several workgroups, and z-chunks when even
// the smallest tile does not.
TileShape default_shape(const Grid &g, int64_t nst, int compute) {
    static const int pref[][3] = {{32, 16, 2}, {32, 8, 2}, {16, 8, 1}};
    static const int pref32[][3] = {{32, 16, 2}, {32, 8, 2}, {16, 8, 1}};
    TileShape sh{1, 16, 8, 0};
    sh.PD = 1;
    for (const auto &c : (compute == 0 ? pref : pref32)) {
        const int64_t tiles = (int64_t)((g.n[0] + c[0] - 1) / c[0]) * ((g.n[1] + c[1] - 1) / c[1]);
        sh.TX = c[0];
        sh.TY = c[1];
        sh.PD = c[2];
        if (tiles * std::max<int64_t>(nst, 1) >= 2048) break;
    }
    sh.BO = 1;
    sh.ZC = g.n[2];
    // a grid with too few tiles to give every compute unit a few workgroups
    // is also split along z, down to chunks of 2 planes (each chunk re-reads
    // 8 planes, which such small batches find in cache)
    const int64_t tiles = (int64_t)((g.n[0] + sh.TX - 1) / sh.TX) * ((g.n[1] + sh.TY - 1) / sh.TY);
    const int64_t wgs = tiles * std::max<int64_t>(nst, 1);
    if (wgs < 1024) sh.ZC = std::max<int>(2, (int)((int64_t)g.n[2] * wgs / 1024));
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
    p.items = plan ? plan->items : nullptr;
    p.rows = g.rows;
    p.zeros = g.zeros;
    p.V = a.compute == 0 ? (const void *)H.V : (const void *)H.V32;
    p.field_dev = a.field_dev;
    p.mask = a.mask;
    p.pair_y = a.pair_y;
    p.pair_out = a.pair_out;
    p.nst = a.nst;
    p.ldp = a.ldp;
    p.np = g.np;
    p.Vim = H.vim;
    if (H.cs_theta != 0) {
        // kin e^{-2 i theta}
        p.kin_h2 = H.kin * std::cos(2.0 * H.cs_theta) / (g.h * g.h);
        p.kin_h2_im = -H.kin * std::sin(2.0 * H.cs_theta) / (g.h * g.h);
    } else {
        p.kin_h2 = H.kin / (g.h * g.h);
        p.kin_h2_im = 0.0;
    }
    p.field = a.field;
    p.h = g.h;
    // box centre along the field axis (one scalar, so that a register copy
    // of these parameters needs no indexed private-memory array)
    p.off_axis = H.axis >= 0 ? 0.5 * (double)(g.n[H.axis] - 1) : 0.0;
    p.cre = a.cre;
    p.cim = a.cim;
    p.nitems = plan ? plan->nitems : 0;
    p.block_order = shape.BO;
    p.ny = g.n[1];
    p.nz = g.n[2];
    p.axis = H.axis;
    p.align = g.align;
    return p;
}

TileShape launch_shape(const Ham &H, const TileShape &tile) {
    TileShape shape = tile;
    if (H.complex_scaled()) {
        bool have = false;
#define RSG_CS_HAVE(X_, Y_, D_) have = have || (shape.TX == X_ && shape.TY == Y_);
        RSG_CS_SHAPES(RSG_CS_HAVE)
#undef RSG_CS_HAVE
        shape.PD = 1;
        if (!have) {
            shape.TX = 16;
            shape.TY = 8;
        }
    }
    if (shape.ZC <= 0) shape.ZC = H.g->n[2];
    return shape;
}

int64_t stencil_blocks(const Ham &H, int64_t nst, int compute, hipStream_t s) {
    int err = RSG_OK;
    const TilePlan *plan = H.g->plan(launch_shape(H, H.tile_for(nst, compute)), s, &err);
    if (!plan) return err;
    return (int64_t)plan->nitems * nst;
}

int launch_stencil(const Ham &H, const StageArgs &a, const TileShape &tile, hipStream_t s) {
    const Grid &g = *H.g;
    int err = RSG_OK;
    const bool cs = H.complex_scaled();
    if (cs && a.compute != 0) {
        set_error("stencil: a complex-scaled Hamiltonian needs the FP64 path");
        return RSG_EUNSUPPORTED;
    }
    const TileShape shape = launch_shape(H, tile);
    const TilePlan *plan = const_cast<Grid &>(g).plan(shape, s, &err);
    if (!plan) return err;
    if (plan->nitems == 0 || a.nst == 0) return RSG_OK;
    if (g.np >= (int64_t)(OOB / 16)) {
        set_error("stencil: grids of 2^27 points or more are not supported");
        return RSG_EUNSUPPORTED;
    }
    const KParams p = make_params(H, a, shape, plan);
    const int64_t nb64 = (int64_t)plan->nitems * a.nst;
    if (nb64 > INT32_MAX) {
        set_error("stencil launch too large");
        return RSG_EUNSUPPORTED;
    }
    const int nb = (int)nb64;
    // an output that no cache level holds is streamed past L2
    const bool nt = (double)a.nst * (double)g.np * (a.out_t == 0 ? 16.0 : 8.0) >= kNtStoreBytes;
    timing_before(s);
    const int rc =
        nt ? stencil_dispatch<true>(a, p, shape, cs, nb, s) : stencil_dispatch<false>(a, p, shape, cs, nb, s);
    timing_after(s);
    if (rc == RSG_EUNSUPPORTED) {
        set_error("stencil: unsupported tile %dx%dx%d depth %d for this precision", shape.B, shape.TX,
                  shape.TY, shape.PD);
        return rc;
    }
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

int stencil_batch_grid(const TileShape &shape, bool first, bool nt) {
    return nt ? batch_dispatch<true>(shape, first, nullptr, nullptr, nullptr, 0, 0.0, 0.0, nullptr, -1, nullptr)
              : batch_dispatch<false>(shape, first, nullptr, nullptr, nullptr, 0, 0.0, 0.0, nullptr, -1, nullptr);
}

int launch_stencil_batch(const TileShape &shape, int mode, bool first, bool nt, const KParams *sysp,
                         const BatchItem *items, const int32_t *seg, int32_t nitems, double cre, double cim,
                         int32_t *ctr, int grid, hipStream_t s) {
    if (nitems == 0) return RSG_OK;
    if (mode != 1) {
        set_error("batched stencil: only Horner stages are batched");
        return RSG_EUNSUPPORTED;
    }
    if (grid <= 0 || !ctr || !seg) {
        set_error("batched stencil: need a persistent grid size > 0, work counters and segment bounds");
        return RSG_EINVAL;
    }
    timing_before(s);
    const int rc = nt ? batch_dispatch<true>(shape, first, sysp, items, seg, nitems, cre, cim, ctr, grid, s)
                      : batch_dispatch<false>(shape, first, sysp, items, seg, nitems, cre, cim, ctr, grid, s);
    timing_after(s);
    if (rc != RSG_OK) {
        if (rc == RSG_EUNSUPPORTED)
            set_error("batched stencil: unsupported tile %dx%dx%d depth %d", shape.B, shape.TX, shape.TY, shape.PD);
        return rc;
    }
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}

}  // namespace rsg
