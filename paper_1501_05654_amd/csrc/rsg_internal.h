// Internal declarations shared by the HIP translation units of librsg.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "rsg.h"

namespace rsg {

// ---------------------------------------------------------------- errors --

void set_error(const char *fmt, ...);
void clear_error();

#define RSG_CHECK_HIP(expr)                                                        \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::rsg::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                             __FILE__, __LINE__);                                  \
            return RSG_EHIP;                                                       \
        }                                                                          \
    } while (0)

#define RSG_REQUIRE(cond, code, ...)      \
    do {                                  \
        if (!(cond)) {                    \
            ::rsg::set_error(__VA_ARGS__); \
            return (code);                \
        }                                 \
    } while (0)

// Run a body that may throw (host allocation) and convert to an error code.
template <class F>
int guarded(F &&f) {
    try {
        return f();
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return RSG_ENOMEM;
    } catch (...) {
        set_error("unexpected host exception");
        return RSG_EINVAL;
    }
}

// ----------------------------------------------------------- launch plan --

// Tile shape of the z-marching stencil: B orbitals (only B = 1 is compiled) x TX x
// TY columns per workgroup, marching along z in chunks of at most ZC planes.
// PD is the software-pipeline depth (planes in flight: 1..2; 0 selects the
// lean march).  PT = 1 launches the tiles of a z-chunk in Morton order;
// PT > 1 groups tiles into PT x PT patches that share one z-range and are
// launched consecutively.  BO is the block order (0: orbital fastest,
// 1: orbital slowest).  ZM = 1 marches from the box's centre plane outward
// (upward above it, downward below it) with the longest tiles of each
// z-chunk first.  The launch plan depends on (TX, TY, ZC, PT, ZM).
struct TileShape {
    int B, TX, TY, ZC;
    int PD = 1;
    int PT = 0;
    int BO = 0;  // block order: 0 = orbital fastest, 1 = orbital slowest, G >= 2 = groups of G orbitals
    int ZM = 0;  // z-march: 0 = upward from each tile's lowest plane, 1 = outward from the centre
    bool operator<(const TileShape &o) const {
        if (B != o.B) return B < o.B;
        if (TX != o.TX) return TX < o.TX;
        if (TY != o.TY) return TY < o.TY;
        if (ZC != o.ZC) return ZC < o.ZC;
        if (PD != o.PD) return PD < o.PD;
        if (PT != o.PT) return PT < o.PT;
        if (BO != o.BO) return BO < o.BO;
        return ZM < o.ZM;
    }
};

// Work items of one tile shape on one grid: (tx, ty, zs, ze) per item: the
// tile marches over planes zs, zs + dir, ... up to ze exclusive, dir = +1 if
// ze > zs, else -1.
struct TilePlan {
    int4 *items = nullptr;  // device
    int32_t nitems = 0;
};

// ------------------------------------------------------------------ grid --

struct Grid {
    int32_t shape = 0;
    int32_t n[3] = {0, 0, 0};  // tight box x, y, z
    int64_t np = 0;            // slots per field: box points, plus dead slots when align > 1
    int64_t npts = 0;          // box points
    int32_t align = 1;         // row bases are multiples of align (a power of two)
    double h = 0;
    // rows[z*ny + y] = {base, x0 | x1 << 16}: point (x,y,z) is in the box iff
    // x0 <= x < x1, with compact index base + x; a non-empty row owns the
    // slots base + x for x in [x0, x1) widened to multiples of align.
    int2 *rows = nullptr;       // device [ny*nz + 1]; entry ny*nz is an empty row
    double *zeros = nullptr;    // device, 256 zero bytes: target of masked-off loads
    std::vector<int2> rows_host;
    int32_t *ijk = nullptr;     // device [np][3]
    std::map<TileShape, TilePlan> plans;
    ~Grid();
    const TilePlan *plan(const TileShape &s, hipStream_t stream, int *err);
};

// ----------------------------------------------------------- Hamiltonian --

struct Ham {
    Grid *g = nullptr;
    double kin = -0.5;
    int32_t axis = -1;
    double *V = nullptr;     // device [np] or null
    float *V32 = nullptr;    // device [np] FP32 copy or null
    double *mask = nullptr;  // device [np] absorber mask applied after every step, or null
    // complex scaling r -> r e^{i theta}: kinetic prefactor kin e^{-2 i theta}
    // and an imaginary part of the local potential (device [np] or null)
    double cs_theta = 0;
    double *vim = nullptr;
    bool complex_scaled() const { return cs_theta != 0 || vim != nullptr; }
    // projectors, padded per atom to a multiple of 16 support entries
    int32_t natoms = 0;
    int32_t *kb_idx = nullptr;   // device [total_padded]
    double *kb_p = nullptr;      // device [total_padded][4]
    float *kb_p32 = nullptr;     // device FP32 copy
    double *kb_E = nullptr;      // device [natoms][4]
    std::vector<int64_t> kb_off; // host [natoms+1] padded offsets
    std::vector<int64_t> kb_len; // host [natoms] true support sizes
    int4 *gather_items = nullptr;   // device: one per atom {offset, padded length, length, atom}
    // scatter work: per colour a device list of {atom, entry0} (16 entries each)
    std::vector<int2 *> scatter_items;
    std::vector<int32_t> scatter_counts;
    // stencil tile shape per (nst, compute) chosen by rsg_autotune / rsg_set_tile
    std::map<std::pair<int64_t, int>, TileShape> tiles;
    TileShape tile_for(int64_t nst, int compute) const;
    ~Ham();
};

// ------------------------------------------------------------ complex ----

template <class T> struct cpx;
template <> struct cpx<double> { using type = double2; };
template <> struct cpx<float> { using type = float2; };

// ------------------------------------------------------------ launchers --

// Stencil stage: out = [base +] c * (kin Lap + V + field x_axis)(in).
// mode 0: out = H in (no base, c = 1).  mode 1: out = base + c H in.
// in_t / out_t: 0 = complex128, 1 = complex64.  compute: 0 = FP64, 1 = FP32.
// All operands are orbital-major with ldp complex values between orbitals;
// base is always complex128.
struct StageArgs {
    const void *in = nullptr;
    const void *base = nullptr;
    void *out = nullptr;
    int in_t = 0, out_t = 0, compute = 0, mode = 0;
    bool first = false;  // base == in (every stage but the last of a mixed or masked step)
    const double *mask = nullptr;  // mode 1: out = mask * (base + c H in)
    // Adjoint pair (first-type FP64 stages only): with pair_y set, the stage
    // also sums conj(in) x_axis pair_y over the points it computes, one
    // complex partial per workgroup, written to pair_out at the workgroup's
    // place in the launch order (stencil_blocks entries).
    const void *pair_y = nullptr;
    double *pair_out = nullptr;
    int64_t nst = 0, ldp = 0;
    double field = 0;
    const double *field_dev = nullptr;
    double cre = 1, cim = 0;
};
// Kernel parameters of one stencil stage on one system (also stored in
// device memory, one per system, by the batched path).
struct KParams {
    const void *in;
    const void *base;
    void *out;
    const int4 *items;
    const int2 *rows;
    const double *zeros;
    const void *V;
    const double *field_dev;
    const double *mask;
    const double *Vim;  // imaginary part of the local potential (complex scaling) or null
    const void *pair_y; // adjoint pair operand, or null
    double *pair_out;   // adjoint pair partials [blocks][2]
    int64_t nst, ldp, np;
    double kin_h2;
    double kin_h2_im;   // imaginary part of the kinetic prefactor over h^2 (complex scaling)
    double field;
    double h;
    double off_axis;    // box centre along the field axis, in grid steps
    double cre, cim;
    int32_t nitems;
    int32_t block_order;
    int32_t ny, nz;
    int32_t axis;
    int32_t align;  // row alignment of the grid (1: compact rows, no dead slots)
};
// Stage outputs of at least this many bytes (the size of the last-level
// cache behind L2) are written with non-temporal stores.
constexpr double kNtStoreBytes = 256.0 * 1024 * 1024;
// One work item of the batched stencil: tile (tx, ty, z0, z1) of system sys,
// orbital ob.
struct BatchItem {
    int4 tile;
    int32_t sys, ob;
};
KParams make_params(const Ham &H, const StageArgs &a, const TileShape &shape, const TilePlan *plan);
int launch_stencil(const Ham &H, const StageArgs &a, const TileShape &shape, hipStream_t s);
// The tile shape a stencil launch of H really runs for the requested one:
// complex-scaled Hamiltonians have kernels for a few depth-1 shapes only
// (another depth maps to depth 1 of the same tile, another tile to 16 x 8);
// ZC = 0 becomes the whole z-extent.
TileShape launch_shape(const Ham &H, const TileShape &tile);
// Workgroups of one stencil launch of nst orbitals with H's tile for this
// precision (the number of pair partials of an adjoint stage), or a negative
// error code.  May create the tile's launch plan (not during capture).
int64_t stencil_blocks(const Ham &H, int64_t nst, int compute, hipStream_t s);
// Work queues of the batched stencil: one per XCD of the device.
constexpr int kBatchQueues = 8;
// seg: kBatchQueues + 1 device int32 bounds, segment q of the item list is
// [seg[q], seg[q + 1]) with seg[0] = 0 and seg[kBatchQueues] = nitems.
// ctr: kBatchQueues + 1 device int32 work counters, zero before the first
// launch (each launch leaves them zero again); launches sharing them must
// not overlap.  nt: the kernel set with non-temporal output stores.
int launch_stencil_batch(const TileShape &shape, int mode, bool first, bool nt, const KParams *sysp,
                         const BatchItem *items, const int32_t *seg, int32_t nitems, double cre, double cim,
                         int32_t *ctr, int grid, hipStream_t s);
// Resident workgroups of the batched kernel for this shape (or an error code).
int stencil_batch_grid(const TileShape &shape, bool first, bool nt);
TileShape default_shape(const Grid &g, int64_t nst, int compute);
std::vector<TileShape> tile_candidates(int compute);

// KB projectors.  gather: D[a][i][col] = h^3 sum_e p[e][i] in(idx[e], col)
// (col over the 2*nst real columns: re and im of each orbital); scatter:
// out(idx[e], col) += sum_i p[e][i] (c E_i D[a][i][.])[col], times mask(idx[e])
// when a mask is given.  Operands are orbital-major with ldp complex values
// between orbitals.
int launch_kb_gather(const Ham &H, const void *in, int in_t, int compute, int64_t nst, int64_t ldp,
                     void *D, hipStream_t s);
int launch_kb_scatter(const Ham &H, void *out, int out_t, int compute, int64_t nst, int64_t ldp,
                      const void *D, double cre, double cim, const double *mask, hipStream_t s);
size_t kb_workspace_bytes(const Ham &H, int64_t nst);

// Per-system projector parameters of one stage of the batched path (FP64).
struct KbSys {
    const double *in;   // gather input (complex as pairs of doubles)
    double *out;        // scatter output
    int64_t ldo, ncols; // 2*ldp (doubles between orbitals), 2*nst
    const int4 *atoms;  // {offset, padded length, length, atom}
    const int32_t *idx;
    const double *p;
    const double *E;
    double *D;          // [natoms][4][ncols]
    double *P;          // [natoms][4][nchunk][ncols] support-chunk partials (nchunk > 1)
    int32_t nchunk, natoms;
    double h3;
};
// Support chunks of the projector gather for a batch of nst orbitals (the
// single-system and batched paths use the same split, so they agree bit
// for bit); the partials live in the projector workspace behind D.
int gather_chunks(const Ham &H, int64_t nst);
size_t gather_partials_offset(const Ham &H, int64_t nst);
// items {system, atom, column tile, chunk}
int launch_kb_gather_batch(const KbSys *sys, const int4 *items, int32_t nitems, hipStream_t s);
// items {system, block of 256 D entries}: D = h3 * sum of the chunk partials
int launch_kb_gather_sum_batch(const KbSys *sys, const int2 *items, int32_t nitems, hipStream_t s);
int launch_kb_scatter_batch(const KbSys *sys, const int4 *items, int32_t nitems, double cre, double cim,
                            hipStream_t s);

// Bump allocator over a caller-provided workspace (256-byte aligned pieces).
struct Carve {
    char *base;
    size_t cap, used = 0;
    bool ok = true;
    Carve(void *p, size_t n) : base((char *)p), cap(n) {}
    void *take(size_t n) {
        const size_t a = (used + 255) & ~(size_t)255;
        if (a + n > cap || (!base && n)) {
            ok = false;
            return nullptr;
        }
        used = a + n;
        return base + a;
    }
    // everything that is left (aligned); *n receives its size
    void *take_rest(size_t *n) {
        const size_t a = (used + 255) & ~(size_t)255;
        if (!base || a >= cap) {
            ok = false;
            *n = 0;
            return nullptr;
        }
        *n = cap - a;
        used = cap;
        return base + a;
    }
};

inline size_t rounded(size_t n) { return (n + 255) & ~(size_t)255; }

// Bytes of an orbital-major batch of nst orbitals with stride ldp.
inline size_t batch_bytes(int64_t nst, int64_t ldp, size_t elem) { return (size_t)nst * (size_t)ldp * elem; }

// Argument checks shared by the entry points that take an orbital-major
// batch [nst][ldp] (RSG_EINVAL / RSG_ESHAPE with a message).
int check_batch(const Ham *H, const void *p, int64_t nst, int64_t ldp, const char *who);
// out = H(in) for an FP64 orbital-major batch; D: kb_workspace_bytes(H, nst).
int hpsi_impl(const Ham &H, const void *in, void *out, int64_t nst, int64_t ldp, double field,
              const double *field_dev, void *D, hipStream_t s);
// The four roots of the Taylor(4) polynomial sum_{k<=4} z^k/k!, largest
// modulus first ({re, im} pairs), and whether a step of this handle in dtype
// runs as the product of their linear factors (else as 1 + z times the
// product of the cubic tail's factors).
const std::complex<double> *taylor4_roots();
bool step_is_product(const Ham &H, int32_t dtype);

// Reductions: partial sums per block then a fixed-order final pass.
// kind 0: <a|b> (complex out [2*nst]); 1: |a|^2 (out [nst]);
// 2: x_axis |a|^2 (out [nst]); 3: sum a b without conjugation (complex out
// [2*nst]); all scaled by h^3.  Operands orbital-major.
size_t reduce_workspace_bytes(const Grid &g, int64_t nst);
int launch_reduce(const Grid &g, int kind, int axis, const double2 *a, const double2 *b,
                  int64_t nst, int64_t ldp, double *out, void *ws, size_t ws_bytes, hipStream_t s);

// Pointwise helpers.
int launch_mul_axis(const Grid &g, int axis, const double2 *src, double2 *dst, int64_t nst,
                    int64_t ldp, hipStream_t s);
// g = 2 Re sum_{k=1}^{4} a[k-1] h3 sum_b P[k-1][b] over the pair partials
// P[4][nb] (complex) of the four adjoint stages, summed in a fixed order.
int launch_pair_final(const double *P, int64_t nb, const double2 a[4], double h3, double *g, hipStream_t s);
int launch_accumulate(const double *src, double *dst, hipStream_t s);

// Kernel timing hooks around stencil launches.
void timing_before(hipStream_t s);
void timing_after(hipStream_t s);

}  // namespace rsg

struct rsg_grid_s : rsg::Grid {};
struct rsg_ham_s : rsg::Ham {};
