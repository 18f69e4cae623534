// Grid setup: box membership, compact numbering and stencil launch plans.
//
// A field on the grid is a linear array over the points of the simulation
// box, with the grid structure kept separately (section "Parallelization,
// optimizations and graphics processing units").  The structure kept here is
// one entry per (y, z) row of the tight bounding box: the x-range of the row
// inside the box and the compact index of its first point.  Compact order is
// z-major, then y, then x, so every row is contiguous in memory and a point's
// index is rows[z*ny + y].base + x.
//
// Row-aligned grids (align A > 1, a power of two) keep the same order but
// give each non-empty row the slots of its x-range widened to multiples of
// A (base a multiple of A).  A tile's row segment, which starts at a
// multiple of the tile width, then starts on a memory line.  The extra
// "dead" slots hold no point: their coordinates read -1, the stencil writes
// zero there and never reads them.
#include "rsg_internal.h"

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstring>

namespace rsg {

namespace {

__device__ int64_t isqrt_dev(int64_t q) {
    int64_t m = (int64_t)sqrt((double)q);
    while ((m + 1) * (m + 1) <= q) ++m;
    while (m * m > q) --m;
    return m;
}

// Row extents: sphere rows hold the x with (x-M)^2 <= Q - (y-M)^2 - (z-M)^2.
__global__ void k_row_extent(int shape, int32_t nx, int32_t ny, int32_t nz, int64_t Q, int32_t M,
                             int32_t *x0, int32_t *len) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (int64_t)ny * nz) return;
    const int64_t y = r % ny, z = r / ny;
    if (shape == RSG_BOX_SPHERE) {
        const int64_t dy = y - M, dz = z - M;
        const int64_t rem = Q - dy * dy - dz * dz;
        if (rem < 0) {
            x0[r] = 0;
            len[r] = 0;
        } else {
            const int64_t xm = isqrt_dev(rem);
            x0[r] = (int32_t)(M - xm);
            len[r] = (int32_t)(2 * xm + 1);
        }
    } else {
        x0[r] = 0;
        len[r] = nx;
    }
}

// Slots a row takes: its x-range [a, a + l) widened to multiples of A.
__device__ __forceinline__ int64_t row_slots(int32_t a, int32_t l, int32_t A) {
    return l > 0 ? (int64_t)(((a + l + A - 1) & -A) - (a & -A)) : 0;
}

// Exclusive scan of the row slot counts in one workgroup (fixed order): each
// thread sums a contiguous chunk, the 1024 chunk totals are scanned in LDS,
// then each thread writes its rows.  Writes rows[] and the total.
__global__ void __launch_bounds__(1024) k_row_scan(const int32_t *x0, const int32_t *len,
                                                   int64_t nrows, int32_t A, int2 *rows, int64_t *total) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (nrows + 1023) / 1024;
    const int64_t r0 = t * chunk, r1 = min(nrows, r0 + chunk);
    int64_t s = 0;
    for (int64_t r = r0; r < r1; ++r) s += row_slots(x0[r], len[r], A);
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t start = t == 0 ? 0 : part[t - 1];
    for (int64_t r = r0; r < r1; ++r) {
        const int32_t a = x0[r], l = len[r];
        rows[r] = make_int2((int32_t)(start - (a & -A)), a | ((a + l) << 16));
        start += row_slots(a, l, A);
    }
    if (t == 1023) *total = part[1023];
}

// Box coordinates of every compact point, one thread per (row, x).
__global__ void k_coords(const int2 *rows, int32_t nx, int32_t ny, int64_t nrows, int32_t *ijk) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nrows * nx) return;
    const int64_t r = g / nx;
    const int32_t x = (int32_t)(g % nx);
    const int2 row = rows[r];
    const int32_t a = row.y & 0xffff, b = (row.y >> 16) & 0xffff;
    if (x < a || x >= b) return;
    const int64_t p = (int64_t)row.x + x;
    ijk[3 * p + 0] = x;
    ijk[3 * p + 1] = (int32_t)(r % ny);
    ijk[3 * p + 2] = (int32_t)(r / ny);
}

}  // namespace

Grid::~Grid() {
    for (auto &kv : plans)
        if (kv.second.items) (void)hipFree(kv.second.items);
    if (rows) (void)hipFree(rows);
    if (zeros) (void)hipFree(zeros);
    if (ijk) (void)hipFree(ijk);
}

// Work items for one tile shape: every (tx, ty) tile that holds box points,
// with its z-extent split into chunks of at most ZC planes.  Within a chunk
// the tiles follow row order (PT = 0: ty, then tx) or the Morton (Z-curve)
// order of (tx, ty) (PT = 1).
//   ZM = 0: chunks start at each tile's lowest plane and march upward; items
//     are ordered chunk-major.
//   ZM = 1: chunks are aligned to the box's centre plane zc = nz / 2; planes
//     >= zc march upward from zc, planes < zc downward from zc - 1, chunk by
//     chunk outward (up-chunk j, then down-chunk j), and within a chunk the
//     tiles with the most planes come first.  Tiles resident together then
//     start on the same plane and advance together, so neighbours read each
//     other's planes from L2 while they are still there.
//   ZM = 2: chunks are aligned to multiples of ZC in z (the same planes for
//     every tile), items chunk-major and in tile order within a chunk.
//     Workgroups launched together then march the same planes side by side,
//     so each reads its halo lines while its neighbours' own loads of those
//     lines are still in L2.
//   PT >= 2 (with ZM = 0): tiles are grouped into PT x PT patches; all tiles
//     of a patch march over the patch's common z-extent, and items are ordered
//     patch-major, then chunk, then tile.
const TilePlan *Grid::plan(const TileShape &s, hipStream_t stream, int *err) {
    TileShape key{0, s.TX, s.TY, s.ZC};
    key.PD = 0;
    key.PT = s.PT;
    key.ZM = s.ZM;
    auto it = plans.find(key);
    if (it != plans.end()) return &it->second;
    const int nx = n[0], ny = n[1], nz = n[2];
    // A tile covers a row wherever the row owns slots: its x-range widened to
    // multiples of the alignment, so that the stencil writes the zeros of
    // every dead slot (the widened end may pass the box's last column).
    const int A = align;
    int xend = nx;
    for (const int2 &r : rows_host) {
        const int a = r.y & 0xffff, b = (r.y >> 16) & 0xffff;
        if (a < b) xend = std::max(xend, (b + A - 1) & -A);
    }
    const int ntx = (xend + s.TX - 1) / s.TX, nty = (ny + s.TY - 1) / s.TY;
    std::vector<int> zlo((size_t)ntx * nty, nz), zhi((size_t)ntx * nty, -1);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            const int2 r = rows_host[(size_t)z * ny + y];
            const int a0 = r.y & 0xffff, b0 = (r.y >> 16) & 0xffff;
            if (a0 >= b0) continue;
            const int a = a0 & -A, b = (b0 + A - 1) & -A;
            const int ty = y / s.TY;
            for (int tx = a / s.TX; tx <= (b - 1) / s.TX; ++tx) {
                const size_t k = (size_t)ty * ntx + tx;
                zlo[k] = std::min(zlo[k], z);
                zhi[k] = std::max(zhi[k], z);
            }
        }
    // non-empty tiles in the order used inside a z-chunk
    std::vector<int> order;
    for (int ty = 0; ty < nty; ++ty)
        for (int tx = 0; tx < ntx; ++tx)
            if (zhi[(size_t)ty * ntx + tx] >= zlo[(size_t)ty * ntx + tx]) order.push_back(ty * ntx + tx);
    if (s.PT == 1) {
        auto spread = [](uint32_t v) {
            uint64_t r = 0;
            for (int b = 0; b < 16; ++b) r |= (uint64_t)((v >> b) & 1u) << (2 * b);
            return r;
        };
        auto key_of = [&](int k) { return spread((uint32_t)(k % ntx)) | (spread((uint32_t)(k / ntx)) << 1); };
        std::stable_sort(order.begin(), order.end(), [&](int p, int q) { return key_of(p) < key_of(q); });
    }
    std::vector<int4> items;
    if (s.ZM == 2) {
        const int L = std::max(1, s.ZC);
        for (int c = 0; c * L < nz; ++c)
            for (const int k : order) {
                const int a = std::max(zlo[k], c * L), b = std::min(zhi[k] + 1, (c + 1) * L);
                if (a < b) items.push_back(make_int4(k % ntx, k / ntx, a, b));
            }
    } else if (s.ZM == 1) {
        const int zc = nz / 2, L = s.ZC;
        const int nup = (nz - zc + L - 1) / L, ndn = (zc + L - 1) / L;
        for (int j = 0; j < std::max(nup, ndn); ++j)
            for (int half = 0; half < 2; ++half) {
                std::vector<int4> chunk;
                for (const int k : order) {
                    const int tx = k % ntx, ty = k / ntx;
                    if (half == 0) {
                        const int a = std::max(zlo[k], zc + j * L), b = std::min(zhi[k] + 1, zc + (j + 1) * L);
                        if (a < b) chunk.push_back(make_int4(tx, ty, a, b));
                    } else {
                        const int hi = std::min(zhi[k], zc - 1 - j * L), lo = std::max(zlo[k], zc - (j + 1) * L);
                        if (hi >= lo) chunk.push_back(make_int4(tx, ty, hi, lo - 1));
                    }
                }
                std::stable_sort(chunk.begin(), chunk.end(), [](const int4 &p, const int4 &q) {
                    return std::abs(p.w - p.z) > std::abs(q.w - q.z);
                });
                items.insert(items.end(), chunk.begin(), chunk.end());
            }
    } else if (s.PT <= 1) {
        int maxchunks = 0;
        for (const int k : order) maxchunks = std::max(maxchunks, (zhi[k] - zlo[k] + s.ZC) / s.ZC);
        for (int c = 0; c < maxchunks; ++c)
            for (const int k : order) {
                const int z0 = zlo[k] + c * s.ZC;
                if (z0 > zhi[k]) continue;
                items.push_back(make_int4(k % ntx, k / ntx, z0, std::min(zhi[k] + 1, z0 + s.ZC)));
            }
    } else {
        const int npx = (ntx + s.PT - 1) / s.PT, npy = (nty + s.PT - 1) / s.PT;
        for (int py = 0; py < npy; ++py)
            for (int px = 0; px < npx; ++px) {
                int plo = nz, phi = -1;
                for (int ty = py * s.PT; ty < std::min(nty, (py + 1) * s.PT); ++ty)
                    for (int tx = px * s.PT; tx < std::min(ntx, (px + 1) * s.PT); ++tx) {
                        const size_t k = (size_t)ty * ntx + tx;
                        if (zhi[k] < zlo[k]) continue;
                        plo = std::min(plo, zlo[k]);
                        phi = std::max(phi, zhi[k]);
                    }
                if (phi < plo) continue;
                for (int z0 = plo; z0 <= phi; z0 += s.ZC)
                    for (int ty = py * s.PT; ty < std::min(nty, (py + 1) * s.PT); ++ty)
                        for (int tx = px * s.PT; tx < std::min(ntx, (px + 1) * s.PT); ++tx) {
                            const size_t k = (size_t)ty * ntx + tx;
                            if (zhi[k] < zlo[k]) continue;
                            items.push_back(make_int4(tx, ty, z0, std::min(phi + 1, z0 + s.ZC)));
                        }
            }
    }
    TilePlan p;
    p.nitems = (int32_t)items.size();
    if (p.nitems > 0) {
        hipError_t e = hipMalloc(&p.items, sizeof(int4) * items.size());
        if (e == hipSuccess)
            e = hipMemcpyAsync(p.items, items.data(), sizeof(int4) * items.size(),
                               hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            set_error("tile plan upload failed: %s", hipGetErrorString(e));
            if (p.items) (void)hipFree(p.items);
            *err = RSG_EHIP;
            return nullptr;
        }
    }
    *err = RSG_OK;
    return &(plans[key] = p);
}

}  // namespace rsg

using namespace rsg;

extern "C" int rsg_grid_create(const rsg_grid_desc *d, void *stream, rsg_grid_t *out) {
    return rsg_grid_create_aligned(d, 1, stream, out);
}

// Builds a grid of the given shape: a sphere (Q, M as above, nx = ny = nz
// = 2M + 1) or a box of nx x ny x nz points.
static int grid_create(int32_t shape, int32_t nx, int32_t ny, int32_t nz, int64_t Q, int32_t M, double h,
                       int32_t align, void *stream, rsg_grid_t *out) {
    return guarded([&]() -> int {
        hipStream_t s = (hipStream_t)stream;
        auto *g = new rsg_grid_s();
        g->shape = shape;
        g->align = align;
        g->n[0] = nx;
        g->n[1] = ny;
        g->n[2] = nz;
        g->h = h;
        const int64_t nrows = (int64_t)ny * nz;
        int32_t *x0 = nullptr, *len = nullptr;
        int64_t *total = nullptr;
        auto fail = [&](hipError_t e) {
            set_error("rsg_grid_create: %s", hipGetErrorString(e));
            if (x0) (void)hipFree(x0);
            if (len) (void)hipFree(len);
            if (total) (void)hipFree(total);
            delete g;
            return RSG_EHIP;
        };
        hipError_t e;
        if ((e = hipMalloc(&x0, sizeof(int32_t) * nrows)) != hipSuccess) return fail(e);
        if ((e = hipMalloc(&len, sizeof(int32_t) * nrows)) != hipSuccess) return fail(e);
        if ((e = hipMalloc(&total, sizeof(int64_t))) != hipSuccess) return fail(e);
        if ((e = hipMalloc(&g->rows, sizeof(int2) * (nrows + 1))) != hipSuccess) return fail(e);
        if ((e = hipMemsetAsync(g->rows + nrows, 0, sizeof(int2), s)) != hipSuccess) return fail(e);
        if ((e = hipMalloc(&g->zeros, 256)) != hipSuccess) return fail(e);
        if ((e = hipMemsetAsync(g->zeros, 0, 256, s)) != hipSuccess) return fail(e);
        const int bs = 256;
        k_row_extent<<<(unsigned)((nrows + bs - 1) / bs), bs, 0, s>>>(shape, nx, ny, nz, Q, M, x0, len);
        k_row_scan<<<1, 1024, 0, s>>>(x0, len, nrows, align, g->rows, total);
        if ((e = hipGetLastError()) != hipSuccess) return fail(e);
        int64_t np = 0;
        if ((e = hipMemcpyAsync(&np, total, sizeof(int64_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
            return fail(e);
        g->rows_host.resize(nrows);
        if ((e = hipMemcpyAsync(g->rows_host.data(), g->rows, sizeof(int2) * nrows,
                                hipMemcpyDeviceToHost, s)) != hipSuccess)
            return fail(e);
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
        if (np >= INT32_MAX) {
            set_error("rsg_grid_create: %lld points exceed the int32 index range", (long long)np);
            (void)hipFree(x0);
            (void)hipFree(len);
            (void)hipFree(total);
            delete g;
            return RSG_EUNSUPPORTED;
        }
        g->np = np;
        g->npts = 0;
        for (const int2 &r : g->rows_host) g->npts += ((r.y >> 16) & 0xffff) - (r.y & 0xffff);
        if ((e = hipMalloc(&g->ijk, sizeof(int32_t) * 3 * (np > 0 ? np : 1))) != hipSuccess)
            return fail(e);
        // dead slots of a row-aligned grid keep coordinates -1
        if (np > g->npts && (e = hipMemsetAsync(g->ijk, 0xff, sizeof(int32_t) * 3 * np, s)) != hipSuccess)
            return fail(e);
        const int64_t work = nrows * nx;
        k_coords<<<(unsigned)((work + bs - 1) / bs), bs, 0, s>>>(g->rows, nx, ny, nrows, g->ijk);
        if ((e = hipGetLastError()) != hipSuccess) return fail(e);
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(e);
        (void)hipFree(x0);
        (void)hipFree(len);
        (void)hipFree(total);
        *out = g;
        return RSG_OK;
    });
}

static int check_align(int32_t align) {
    RSG_REQUIRE(align >= 1 && align <= 64 && (align & (align - 1)) == 0, RSG_EINVAL,
                "rsg_grid_create: align must be a power of two in 1..64");
    return RSG_OK;
}

extern "C" int rsg_grid_create_aligned(const rsg_grid_desc *d, int32_t align, void *stream, rsg_grid_t *out) {
    clear_error();
    RSG_REQUIRE(d && out, RSG_EINVAL, "rsg_grid_create: null argument");
    int rc = check_align(align);
    if (rc) return rc;
    RSG_REQUIRE(d->h > 0 && std::isfinite(d->h), RSG_EINVAL, "rsg_grid_create: h must be > 0");
    RSG_REQUIRE(d->shape == RSG_BOX_CUBE || d->shape == RSG_BOX_SPHERE, RSG_EINVAL,
                "rsg_grid_create: unknown box shape %d", d->shape);
    int64_t Q = 0;
    int32_t M = 0, nx;
    if (d->shape == RSG_BOX_SPHERE) {
        RSG_REQUIRE(d->radius > 0 && std::isfinite(d->radius), RSG_EINVAL,
                    "rsg_grid_create: radius must be > 0");
        const double q = std::floor((d->radius / d->h) * (d->radius / d->h) + 1e-9);
        RSG_REQUIRE(q < 1.0e8, RSG_EINVAL, "rsg_grid_create: sphere too large (R/h > 10^4)");
        Q = (int64_t)q;
        int64_t m = (int64_t)std::sqrt((double)Q);
        while ((m + 1) * (m + 1) <= Q) ++m;
        while (m * m > Q) --m;
        M = (int32_t)m;
        nx = 2 * M + 1;
    } else {
        RSG_REQUIRE(d->n >= 1, RSG_EINVAL, "rsg_grid_create: cube needs n >= 1");
        nx = d->n;
    }
    RSG_REQUIRE(nx < 32768, RSG_EINVAL, "rsg_grid_create: box wider than 32767 points");
    return grid_create(d->shape, nx, nx, nx, Q, M, d->h, align, stream, out);
}

extern "C" int rsg_grid_create_box(int32_t nx, int32_t ny, int32_t nz, double h, int32_t align, void *stream,
                                   rsg_grid_t *out) {
    clear_error();
    RSG_REQUIRE(out, RSG_EINVAL, "rsg_grid_create_box: null argument");
    int rc = check_align(align);
    if (rc) return rc;
    RSG_REQUIRE(h > 0 && std::isfinite(h), RSG_EINVAL, "rsg_grid_create_box: h must be > 0");
    RSG_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1, RSG_EINVAL, "rsg_grid_create_box: need at least 1 point per axis");
    RSG_REQUIRE(nx < 32768 && ny < 32768 && nz < 32768, RSG_EINVAL,
                "rsg_grid_create_box: box wider than 32767 points");
    RSG_REQUIRE((int64_t)nx * ny * nz < ((int64_t)1 << 31), RSG_EINVAL, "rsg_grid_create_box: too many points");
    return grid_create(RSG_BOX_CUBE, nx, ny, nz, 0, 0, h, align, stream, out);
}

extern "C" int rsg_grid_info(rsg_grid_t g, int64_t *np, int32_t dims[3], double *h) {
    clear_error();
    RSG_REQUIRE(g, RSG_EINVAL, "rsg_grid_info: null grid");
    if (np) *np = g->np;
    if (dims) std::memcpy(dims, g->n, sizeof(int32_t) * 3);
    if (h) *h = g->h;
    return RSG_OK;
}

extern "C" int rsg_grid_points(rsg_grid_t g, int64_t *npoints, int32_t *align) {
    clear_error();
    RSG_REQUIRE(g, RSG_EINVAL, "rsg_grid_points: null grid");
    if (npoints) *npoints = g->npts;
    if (align) *align = g->align;
    return RSG_OK;
}

extern "C" int rsg_grid_coords(rsg_grid_t g, int32_t *ijk_host) {
    clear_error();
    RSG_REQUIRE(g && ijk_host, RSG_EINVAL, "rsg_grid_coords: null argument");
    RSG_CHECK_HIP(hipMemcpy(ijk_host, g->ijk, sizeof(int32_t) * 3 * g->np, hipMemcpyDeviceToHost));
    return RSG_OK;
}

extern "C" int rsg_grid_positions(rsg_grid_t g, double *xyz) {
    clear_error();
    RSG_REQUIRE(g && xyz, RSG_EINVAL, "rsg_grid_positions: null argument");
    return guarded([&]() -> int {
        std::vector<int32_t> ijk((size_t)3 * g->np);
        RSG_CHECK_HIP(hipMemcpy(ijk.data(), g->ijk, sizeof(int32_t) * ijk.size(), hipMemcpyDeviceToHost));
        for (int64_t p = 0; p < g->np; ++p)
            for (int a = 0; a < 3; ++a)
                xyz[3 * p + a] = ijk[3 * p] < 0 ? 0.0  // dead slot of a row-aligned grid
                                                : g->h * ((double)ijk[3 * p + a] - 0.5 * (double)(g->n[a] - 1));
        return RSG_OK;
    });
}

extern "C" int rsg_grid_destroy(rsg_grid_t g) {
    clear_error();
    delete g;
    return RSG_OK;
}
