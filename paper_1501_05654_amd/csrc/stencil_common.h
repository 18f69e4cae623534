// Device helpers of the z-marching stencil kernels: finite-difference
// weights, workgroup-to-XCD remapping, block orders, row-table lookups and
// CDNA buffer loads/stores.
#pragma once

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

// Workgroup b of nb runs on XCD b % 8; give each XCD a contiguous range.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, local = b >> 3;
    return (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + local;
}

// Block order.  Orbital slowest (BO = 1): each XCD sweeps the tiles of one
// orbital at a time, so neighbouring tiles march together and find each
// other's halos and shared row-boundary lines in L2.  Orbital fastest
// (BO = 0): the orbitals of one tile march together and share V and the row
// table in L2.  BO = G >= 2: orbitals in groups of G, each group sweeping
// the tiles with its G orbitals of a tile side by side (V read once per
// group from HBM, neighbouring tiles still resident together).
__device__ __forceinline__ void block_item(const KParams &a, int blk, int *n, int *item) {
    const int nst = (int)a.nst;
    if (a.block_order == 0) {
        *item = blk / nst;
        *n = blk - *item * nst;
    } else if (a.block_order == 1) {
        *n = blk / a.nitems;
        *item = blk - *n * a.nitems;
    } else {
        const int G = a.block_order, per = a.nitems * G;
        const int g = blk / per, r = blk - g * per;
        const int gs = min(G, nst - g * G);  // orbitals in this group
        *item = r / gs;
        *n = g * G + (r - *item * gs);
    }
}

// Branch-free row lookup: an out-of-box row reads the empty sentinel entry
// that follows the table.  Loads are never masked after they return (the
// compiler would place the select where the load is issued and wait there);
// a masked-off lane issues its load at an out-of-range offset, which the
// buffer hardware answers with zero.
// SEL: the test as unsigned compares and selects, which keeps the march's
// step free of branches.
template <bool SEL>
__device__ __forceinline__ int2 row_of(const KParams &a, int y, int z) {
    if constexpr (SEL) {
        const bool v = (unsigned)y < (unsigned)a.ny && (unsigned)z < (unsigned)a.nz;
        return a.rows[v ? z * a.ny + y : a.ny * a.nz];
    } else {
        const bool v = y >= 0 && y < a.ny && z >= 0 && z < a.nz;
        return a.rows[v ? z * a.ny + y : a.ny * a.nz];
    }
}
__device__ __forceinline__ int idx_in_row(int2 r, int x) {
    const int x0 = r.y & 0xffff, x1 = (r.y >> 16) & 0xffff;
    return (x >= x0 && x < x1) ? r.x + x : -1;
}
// Own-column index for loads and the store: a box point gives its index; a
// dead slot of a row-aligned grid (inside the row's x-range widened to
// multiples of align, outside the box) gives -(index) - 2, which every load
// treats as out of range and the store fills with zero; anything else -1.
// SEL as for row_of: selects only.
template <bool SEL>
__device__ __forceinline__ int slot_in_row(int2 r, int x, int align) {
    const int x0 = r.y & 0xffff, x1 = (r.y >> 16) & 0xffff;
    const int a0 = x0 & -align, a1 = (x1 + align - 1) & -align;
    if constexpr (SEL) {
        const int v = r.x + x;
        const bool in = x >= x0 && x < x1, dead = x0 < x1 && x >= a0 && x < a1;
        return in ? v : (dead ? -v - 2 : -1);
    } else {
        if (x >= x0 && x < x1) return r.x + x;
        return (x0 < x1 && x >= a0 && x < a1) ? -(r.x + x) - 2 : -1;
    }
}

// Buffer loads and stores (CDNA): a per-workgroup resource (base address,
// size in bytes) in scalar registers and a 32-bit byte offset per lane.  An
// offset at or beyond the size reads zero and drops a store, in hardware, so
// masked-off lanes need no select and no second address register.
typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef int v2i_t __attribute__((ext_vector_type(2)));
constexpr unsigned OOB = 0x80000000u;    // byte offset beyond every buffer used here
constexpr int RSRC_WORD3 = 0x00020000;   // resource format word of the gfx9 family

// Every operand base and size is the same for all lanes of a workgroup;
// reading them through the first lane tells the compiler so, which keeps
// the resource in scalar registers instead of a per-lane loop around each
// buffer instruction.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, int64_t bytes) {
    const uint64_t u = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    const int nb = __builtin_amdgcn_readfirstlane((int)bytes);
    void *q = (void *)(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(q, (short)0, nb, RSRC_WORD3);
}
template <class T>
__device__ __forceinline__ unsigned boff(int idx) {
    return idx >= 0 ? (unsigned)idx * (unsigned)sizeof(T) : OOB;
}

template <class T> struct BL;
template <> struct BL<double2> {
    static __device__ __forceinline__ double2 ld(__amdgpu_buffer_rsrc_t r, unsigned o) {
        return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)o, 0, 0));
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, unsigned o, double2 v) {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i_t, v), r, (int)o, 0, 0);
    }
    // non-temporal (cache policy NT): the line is not kept in L2
    static __device__ __forceinline__ void st_nt(__amdgpu_buffer_rsrc_t r, unsigned o, double2 v) {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i_t, v), r, (int)o, 0, 2);
    }
};
template <> struct BL<float2> {
    static __device__ __forceinline__ float2 ld(__amdgpu_buffer_rsrc_t r, unsigned o) {
        return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)o, 0, 0));
    }
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, unsigned o, float2 v) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i_t, v), r, (int)o, 0, 0);
    }
    static __device__ __forceinline__ void st_nt(__amdgpu_buffer_rsrc_t r, unsigned o, float2 v) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i_t, v), r, (int)o, 0, 2);
    }
};
template <> struct BL<double> {
    static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, unsigned o) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)o, 0, 0));
    }
};
template <> struct BL<float> {
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, unsigned o) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)o, 0, 0));
    }
};

template <class Tc, class Tin>
__device__ __forceinline__ typename CT<Tc>::c2 load_c(__amdgpu_buffer_rsrc_t r, unsigned o) {
    const Tin v = BL<Tin>::ld(r, o);
    return typename CT<Tc>::c2{(Tc)v.x, (Tc)v.y};
}

// NTS: non-temporal stores, for a stage output much larger than the caches
// (streamed past L2, which then keeps the input planes and the halo lines
// that neighbouring tiles still read); a compile-time choice, since a branch
// per store costs more than the policy gains
template <bool NTS>
__device__ __forceinline__ void store_c(__amdgpu_buffer_rsrc_t r, unsigned o, double2 *, double re, double im) {
    if constexpr (NTS)
        BL<double2>::st_nt(r, o, make_double2(re, im));
    else
        BL<double2>::st(r, o, make_double2(re, im));
}
template <bool NTS>
__device__ __forceinline__ void store_c(__amdgpu_buffer_rsrc_t r, unsigned o, float2 *, double re, double im) {
    if constexpr (NTS)
        BL<float2>::st_nt(r, o, make_float2((float)re, (float)im));
    else
        BL<float2>::st(r, o, make_float2((float)re, (float)im));
}

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }
constexpr int clcm(int a, int b) { return a / cgcd(a, b) * b; }

}  // namespace
}  // namespace rsg
