// Grid-to-memory maps and the generic (gather-form) finite-difference
// Laplacian that works with any of them.
//
// Section "Parallelization, optimizations and graphics processing units"
// (figures gridmaps and gpu_laplacian): a grid function is a linear array,
// the grid structure lives in side tables, and the order in which points are
// stored is free.  Orders that keep grid neighbours close in memory (small
// parallelepiped bricks, a Hilbert curve) make the stencil's neighbour reads
// hit the caches more often than the plain row order.  A map here is such an
// order plus a table of the 24 off-centre stencil neighbours of every point,
// given as positions in the same order; the Laplacian kernel gathers through
// that table and so runs unchanged on every map.
//
// The z-marching stencil of the propagation path does not need any of this:
// it walks rows of the compact order and gets its locality from the tile
// shape.  These maps exist to measure the paper's comparison on MI355X.
#include "rsg_internal.h"

#include <algorithm>
#include <numeric>

namespace rsg {

namespace {

// Workgroup b of nb runs on XCD b % 8; hand each XCD a contiguous range of
// the launch order, so that points close in the map share one L2.
__device__ __forceinline__ int xcd_contiguous(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, local = b >> 3;
    return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + local;
}

constexpr int MB = 256;  // threads per workgroup

// Eighth-order second-derivative weights c_0..c_4 (Fornberg): -205/72, 8/5,
// -1/5, 8/315, -1/560.  Neighbour slot j = 8 axis + k holds the offset
// m = k - 4 for k < 4 and m = k - 3 otherwise, so |m| = 1 + min(3 - k, k - 4).
// One thread per (point, orbital), orbital fastest: a wave reads whole rows
// of nst orbitals of each neighbour.  Taps of equal |m| are summed first
// (x, y, z pairs), then weighted.
__global__ void __launch_bounds__(MB) k_map_lap(const double2 *__restrict__ psi, double2 *__restrict__ out,
                                                const int32_t *__restrict__ nbr, int32_t np, int32_t nst,
                                                int64_t ld, double scale) {
    const int blk = xcd_contiguous(blockIdx.x, gridDim.x);
    const int g = blk * MB + (int)threadIdx.x;
    const int p = g / nst;
    if (p >= np) return;
    const int n = g - p * nst;
    const double2 c = psi[(int64_t)p * ld + n];
    double sr[4] = {0, 0, 0, 0}, si[4] = {0, 0, 0, 0};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = nbr[(int64_t)(8 * a + k) * np + p];
            const int dm = k < 4 ? 3 - k : k - 4;  // |m| - 1
            if (q >= 0) {
                const double2 v = psi[(int64_t)q * ld + n];
                sr[dm] += v.x;
                si[dm] += v.y;
            }
        }
    }
    const double c0 = -205.0 / 72.0, c1 = 8.0 / 5.0, c2 = -1.0 / 5.0, c3 = 8.0 / 315.0, c4 = -1.0 / 560.0;
    const double lr = 3.0 * c0 * c.x + c1 * sr[0] + c2 * sr[1] + c3 * sr[2] + c4 * sr[3];
    const double li = 3.0 * c0 * c.y + c1 * si[0] + c2 * si[1] + c3 * si[2] + c4 * si[3];
    out[(int64_t)p * ld + n] = make_double2(scale * lr, scale * li);
}

// 3D Hilbert index of box coordinates (X[0], X[1], X[2]), each below 2^b,
// after Skilling's axes-to-transpose transform: from the top bit level down,
// each level's lower bits are inverted or exchanged with axis 0 depending on
// the bit of each axis at that level, the result is Gray-coded across the
// axes, and the index is the bits read level by level with axis 0 first.
uint64_t hilbert_index(uint32_t X0, uint32_t X1, uint32_t X2, int b) {
    uint32_t X[3] = {X0, X1, X2};
    const uint32_t top = 1u << (b - 1);
    for (uint32_t Q = top; Q > 1; Q >>= 1) {
        const uint32_t low = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= low;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & low;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t flip = 0;
    for (uint32_t Q = top; Q > 1; Q >>= 1)
        if (X[2] & Q) flip ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= flip;
    uint64_t h = 0;
    for (int lev = b - 1; lev >= 0; --lev)
        for (int i = 0; i < 3; ++i) h = (h << 1) | ((X[i] >> lev) & 1u);
    return h;
}

}  // namespace

}  // namespace rsg

using namespace rsg;

struct rsg_map_s {
    const Grid *g = nullptr;
    int32_t kind = 0, param = 0;
    std::vector<int32_t> order;  // host [np]: compact index of the i-th point in map order
    int32_t *nbr = nullptr;      // device [24][np]: map position of each neighbour, -1 outside
    ~rsg_map_s() {
        if (nbr) (void)hipFree(nbr);
    }
};

extern "C" int rsg_map_create(rsg_grid_t g, int32_t kind, int32_t param, rsg_map_t *out) {
    clear_error();
    RSG_REQUIRE(g && out, RSG_EINVAL, "rsg_map_create: null argument");
    RSG_REQUIRE(kind == RSG_MAP_STANDARD || kind == RSG_MAP_BRICKS || kind == RSG_MAP_HILBERT, RSG_EINVAL,
                "rsg_map_create: unknown map kind %d", kind);
    RSG_REQUIRE(kind != RSG_MAP_BRICKS || (param >= 1 && param <= 64), RSG_EINVAL,
                "rsg_map_create: brick edge must be 1..64 (got %d)", param);
    RSG_REQUIRE(g->np > 0, RSG_EINVAL, "rsg_map_create: empty grid");
    RSG_REQUIRE(g->align == 1, RSG_EUNSUPPORTED, "rsg_map_create: needs a grid with compact rows (align 1)");
    return guarded([&]() -> int {
        const int64_t np = g->np;
        const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
        // box coordinates of every compact point, from the row table
        std::vector<int32_t> cx(np), cy(np), cz(np);
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y) {
                const int2 r = g->rows_host[(size_t)z * ny + y];
                const int x0 = r.y & 0xffff, x1 = (r.y >> 16) & 0xffff;
                for (int x = x0; x < x1; ++x) {
                    const int64_t c = (int64_t)r.x + x;
                    cx[c] = x;
                    cy[c] = y;
                    cz[c] = z;
                }
            }
        auto compact = [&](int x, int y, int z) -> int64_t {
            if (y < 0 || y >= ny || z < 0 || z >= nz || x < 0 || x >= nx) return -1;
            const int2 r = g->rows_host[(size_t)z * ny + y];
            const int x0 = r.y & 0xffff, x1 = (r.y >> 16) & 0xffff;
            return (x >= x0 && x < x1) ? (int64_t)r.x + x : -1;
        };
        auto *m = new rsg_map_s();
        m->g = g;
        m->kind = kind;
        m->param = param;
        m->order.resize(np);
        std::iota(m->order.begin(), m->order.end(), 0);
        if (kind != RSG_MAP_STANDARD) {
            std::vector<uint64_t> key(np);
            if (kind == RSG_MAP_BRICKS) {
                const uint64_t b = (uint64_t)param;
                const uint64_t nbx = (nx + b - 1) / b, nby = (ny + b - 1) / b;
                for (int64_t c = 0; c < np; ++c) {
                    const uint64_t x = cx[c], y = cy[c], z = cz[c];
                    const uint64_t brick = ((z / b) * nby + y / b) * nbx + x / b;
                    key[c] = ((brick * b + z % b) * b + y % b) * b + x % b;
                }
            } else {
                int bits = 1;
                while ((1 << bits) < std::max(nx, std::max(ny, nz))) ++bits;
                for (int64_t c = 0; c < np; ++c)
                    key[c] = hilbert_index((uint32_t)cx[c], (uint32_t)cy[c], (uint32_t)cz[c], bits);
            }
            // keys are distinct, so the order is fully determined
            std::sort(m->order.begin(), m->order.end(),
                      [&](int32_t a, int32_t b) { return key[a] < key[b]; });
        }
        std::vector<int32_t> pos(np);
        for (int64_t i = 0; i < np; ++i) pos[m->order[i]] = (int32_t)i;
        std::vector<int32_t> nb((size_t)24 * np);
        for (int64_t i = 0; i < np; ++i) {
            const int32_t c = m->order[i];
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < 8; ++k) {
                    const int mm = k < 4 ? k - 4 : k - 3;
                    const int64_t q = compact(cx[c] + (a == 0 ? mm : 0), cy[c] + (a == 1 ? mm : 0),
                                              cz[c] + (a == 2 ? mm : 0));
                    nb[(size_t)(8 * a + k) * np + i] = q < 0 ? -1 : pos[q];
                }
        }
        hipError_t e = hipMalloc(&m->nbr, sizeof(int32_t) * nb.size());
        if (e == hipSuccess) e = hipMemcpy(m->nbr, nb.data(), sizeof(int32_t) * nb.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            set_error("rsg_map_create: %s", hipGetErrorString(e));
            delete m;
            return e == hipErrorOutOfMemory ? RSG_ENOMEM : RSG_EHIP;
        }
        *out = m;
        return RSG_OK;
    });
}

extern "C" int rsg_map_destroy(rsg_map_t m) {
    clear_error();
    delete m;
    return RSG_OK;
}

extern "C" int rsg_map_order(rsg_map_t m, int32_t *order_host) {
    clear_error();
    RSG_REQUIRE(m && order_host, RSG_EINVAL, "rsg_map_order: null argument");
    std::copy(m->order.begin(), m->order.end(), order_host);
    return RSG_OK;
}

extern "C" int rsg_map_laplacian(rsg_map_t m, const void *psi, void *out, int64_t nst, int64_t ld, double scale,
                                 void *stream) {
    clear_error();
    RSG_REQUIRE(m && psi && out, RSG_EINVAL, "rsg_map_laplacian: null argument");
    RSG_REQUIRE(nst >= 1 && ld >= nst, RSG_ESHAPE, "rsg_map_laplacian: need 1 <= nst <= ld (nst=%lld, ld=%lld)",
                (long long)nst, (long long)ld);
    const int64_t np = m->g->np;
    RSG_REQUIRE(np * nst < ((int64_t)1 << 31) - MB, RSG_EUNSUPPORTED,
                "rsg_map_laplacian: np * nst must stay below 2^31");
    const char *a = static_cast<const char *>(psi), *b = static_cast<const char *>(out);
    const int64_t bytes = np * ld * 16;
    RSG_REQUIRE(a + bytes <= b || b + bytes <= a, RSG_EINVAL, "rsg_map_laplacian: psi and out overlap");
    const int64_t threads = np * nst;
    const unsigned nblk = (unsigned)((threads + MB - 1) / MB);
    k_map_lap<<<nblk, MB, 0, (hipStream_t)stream>>>(static_cast<const double2 *>(psi), static_cast<double2 *>(out),
                                                    m->nbr, (int32_t)np, (int32_t)nst, ld, scale);
    RSG_CHECK_HIP(hipGetLastError());
    return RSG_OK;
}
