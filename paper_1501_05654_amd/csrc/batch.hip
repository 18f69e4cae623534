// Many independent systems propagated together.
//
// The paper's basic object is a group of states rather than one state
// (section "Parallelization, optimizations and graphics processing units");
// here the group extends across systems.  The systems are grouped into size
// classes (by the width of their box), each class with its own stencil tile
// shape; every stage of a Taylor(4) step runs, per class, as one persistent
// stencil launch over a list of (system, tile, z-range, orbital) items
// (largest systems first, each sweeping its tiles orbital by orbital; the
// list is cut into one contiguous segment per XCD, so that each XCD's L2
// holds the halos its neighbouring tiles share), preceded by one projector gather launch and followed by one scatter launch
// per colour, all systems at once.  A step sequence can be captured once into
// a HIP graph and replayed.  Each output point is computed by the same
// arithmetic as the single-system path, so the results are bitwise equal to
// propagating each system alone with its class's tile shape.
#include "rsg_internal.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <tuple>

namespace rsg {

// Systems of one size class share a tile shape and a persistent launch per
// stage; the classes of a stage run back to back on the caller's stream.
struct BatchClass {
    TileShape tile{1, 32, 8, 0};
    std::vector<int32_t> sys;    // member systems
    BatchItem *items = nullptr;  // device work list of this class
    int32_t *seg = nullptr;      // device bounds of the list's per-XCD segments
    int32_t nitems = 0;
    int grid = 0;                // resident workgroups of the class's kernel
};

struct Batch {
    std::vector<rsg_system_desc> sys;
    std::vector<void *> w1, w2, D;  // per-system work buffers inside the caller's workspace
    std::vector<BatchClass> cls;
    int32_t grid_cap = 0;  // at most this many persistent workgroups per launch (0: no cap)
    bool nt = false;       // stage outputs written with non-temporal stores
    KParams *sp[4] = {nullptr, nullptr, nullptr, nullptr};  // device, per stage, one per system
    KbSys *kb[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t *ctr = nullptr;  // device work counters of the persistent stencil (zero between launches)
    int4 *gitems = nullptr;
    int32_t ngitems = 0;
    int2 *sumitems = nullptr;  // projector chunk sums {system, block of 256 D entries}
    int32_t nsumitems = 0;
    std::vector<int4 *> sitems;  // scatter items per colour
    std::vector<int32_t> nsitems;
    std::map<std::tuple<double, int64_t, hipStream_t>, hipGraphExec_t> graphs;
    void drop_graphs() {
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
    }
    void free_tables() {
        for (int k = 0; k < 4; ++k) {
            if (sp[k]) (void)hipFree(sp[k]);
            if (kb[k]) (void)hipFree(kb[k]);
            sp[k] = nullptr;
            kb[k] = nullptr;
        }
        for (auto &c : cls) {
            if (c.items) (void)hipFree(c.items);
            if (c.seg) (void)hipFree(c.seg);
            c.items = nullptr;
            c.seg = nullptr;
            c.nitems = 0;
        }
        if (ctr) (void)hipFree(ctr);
        ctr = nullptr;
        if (gitems) (void)hipFree(gitems);
        if (sumitems) (void)hipFree(sumitems);
        sumitems = nullptr;
        nsumitems = 0;
        for (auto *p : sitems)
            if (p) (void)hipFree(p);
        gitems = nullptr;
        sitems.clear();
        nsitems.clear();
        drop_graphs();
    }
    ~Batch() { free_tables(); }
};

// Default size classes: systems whose tight box is narrower than 48 points,
// 48 to 79 points, and 80 points or more (the spheres of radius 4 to 12 bohr
// at h = 0.25 span 33 to 97 points).  A tile that suits the widest spheres
// leaves most lanes of a narrow sphere's tiles idle, and the other way round
// narrow tiles re-read more halo per output on wide spheres.
constexpr int kClassEdges[] = {48, 80};

namespace {

size_t rnd(size_t n) { return (n + 255) & ~(size_t)255; }

size_t sys_bytes(const rsg_system_desc &d) {
    const Ham &H = *d.ham;
    return 2 * rnd((size_t)d.nst * (size_t)d.ldp * 16) + rnd(kb_workspace_bytes(H, d.nst));
}

template <class T>
int upload(T **dst, const std::vector<T> &v, hipStream_t s) {
    if (v.empty()) return RSG_OK;
    RSG_CHECK_HIP(hipMalloc(dst, sizeof(T) * v.size()));
    RSG_CHECK_HIP(hipMemcpyAsync(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
    return RSG_OK;
}

// Stage k (0..3) of a step: in, base, out buffers of system i.  The stages
// run in product form, each its own base (base = in).
void stage_buffers(const Batch &b, size_t i, int k, const void **in, const void **base, void **out) {
    void *psi = b.sys[i].psi;
    switch (k) {
        case 0: *in = psi; *out = b.w1[i]; break;
        case 1: *in = b.w1[i]; *out = b.w2[i]; break;
        case 2: *in = b.w2[i]; *out = b.w1[i]; break;
        default: *in = b.w1[i]; *out = psi; break;
    }
    *base = *in;
}

// Stencil items of class c for its tile: its systems with the most work
// first (the small ones fill the tail of the persistent grid), each system
// sweeping its tiles one orbital at a time so that neighbouring tiles are
// resident together.  Replaces the class's device list.
int build_class(Batch &b, size_t c, hipStream_t s) {
    BatchClass &cl = b.cls[c];
    if (cl.items) (void)hipFree(cl.items);
    if (cl.seg) (void)hipFree(cl.seg);
    cl.items = nullptr;
    cl.seg = nullptr;
    cl.nitems = 0;
    b.drop_graphs();
    std::vector<int32_t> by_work = cl.sys;
    std::stable_sort(by_work.begin(), by_work.end(), [&](int32_t p, int32_t q) {
        return b.sys[p].ham->g->np * b.sys[p].nst > b.sys[q].ham->g->np * b.sys[q].nst;
    });
    std::vector<BatchItem> items;
    int err = RSG_OK;
    for (const int32_t i : by_work) {
        const rsg_system_desc &d = b.sys[i];
        TileShape sh = cl.tile;
        sh.PT = 0;
        sh.BO = 0;
        sh.ZC = sh.ZC > 0 ? sh.ZC : d.ham->g->n[2];  // ZM as chosen for the class
        const TilePlan *plan = d.ham->g->plan(sh, s, &err);
        if (!plan) return err;
        // copy the plan's items back to the host to expand them per orbital
        std::vector<int4> pit(plan->nitems);
        if (plan->nitems)
            RSG_CHECK_HIP(hipMemcpy(pit.data(), plan->items, sizeof(int4) * plan->nitems, hipMemcpyDeviceToHost));
        for (int n = 0; n < (int)d.nst; ++n)
            for (const int4 &t : pit) items.push_back(BatchItem{t, i, n});
    }
    // per-XCD segments of about equal work: a march costs its z-planes plus
    // the planes that fill the register ring
    std::vector<int64_t> cum(items.size() + 1, 0);
    for (size_t w = 0; w < items.size(); ++w)
        cum[w + 1] = cum[w] + std::abs(items[w].tile.w - items[w].tile.z) + 8;
    std::vector<int32_t> seg(kBatchQueues + 1, 0);
    for (int q = 1; q < kBatchQueues; ++q)
        seg[q] = (int32_t)(std::lower_bound(cum.begin(), cum.end(), cum.back() * q / kBatchQueues) - cum.begin());
    seg[kBatchQueues] = (int32_t)items.size();
    for (int q = 1; q <= kBatchQueues; ++q) seg[q] = std::max(seg[q], seg[q - 1]);
    cl.grid = stencil_batch_grid(cl.tile, true, b.nt);
    if (cl.grid <= 0) return cl.grid;
    int rc = upload(&cl.items, items, s);
    if (rc) return rc;
    if ((rc = upload(&cl.seg, seg, s))) return rc;
    cl.nitems = (int32_t)items.size();
    RSG_CHECK_HIP(hipStreamSynchronize(s));
    return RSG_OK;
}

// (Re)build the per-system parameter tables, the projector work lists and
// every class's stencil items.
int build_tables(Batch &b, hipStream_t s) {
    b.free_tables();
    std::vector<int4> gitems;
    std::vector<int2> sumitems;
    std::vector<std::vector<int4>> sitems;
    std::vector<KParams> sp[4];
    std::vector<KbSys> kb[4];
    for (size_t i = 0; i < b.sys.size(); ++i) {
        const rsg_system_desc &d = b.sys[i];
        Ham &H = *d.ham;
        for (int k = 0; k < 4; ++k) {
            StageArgs a;
            stage_buffers(b, i, k, &a.in, &a.base, &a.out);
            a.mode = 1;
            a.nst = d.nst;
            a.ldp = d.ldp;
            a.first = k == 0;
            // the persistent kernel takes its tiles from the class's list,
            // not from a plan
            sp[k].push_back(make_params(H, a, TileShape{1, 32, 8, 0}, nullptr));
            KbSys ks;
            ks.in = (const double *)a.in;
            ks.out = (double *)a.out;
            ks.ldo = 2 * d.ldp;
            ks.ncols = 2 * d.nst;
            ks.atoms = H.gather_items;
            ks.idx = H.kb_idx;
            ks.p = H.kb_p;
            ks.E = H.kb_E;
            ks.D = (double *)b.D[i];
            ks.nchunk = gather_chunks(H, d.nst);
            ks.natoms = H.natoms;
            ks.P = ks.nchunk > 1 ? (double *)((char *)b.D[i] + gather_partials_offset(H, d.nst)) : nullptr;
            ks.h3 = H.g->h * H.g->h * H.g->h;
            kb[k].push_back(ks);
        }
        const int nct = (int)((2 * d.nst + 15) / 16);
        const int nchunk = gather_chunks(H, d.nst);
        for (int a = 0; a < H.natoms; ++a)
            for (int ct = 0; ct < nct; ++ct)
                for (int ch = 0; ch < nchunk; ++ch) gitems.push_back(make_int4((int)i, a, ct, ch));
        if (nchunk > 1) {
            const int64_t nd = (int64_t)H.natoms * 4 * 2 * d.nst;
            for (int64_t blk = 0; blk < (nd + 255) / 256; ++blk) sumitems.push_back(make_int2((int)i, (int)blk));
        }
        if (H.natoms > 0) {
            // host copy of this system's scatter lists, per colour
            for (size_t c = 0; c < H.scatter_items.size(); ++c) {
                if (sitems.size() <= c) sitems.resize(c + 1);
                std::vector<int2> v(H.scatter_counts[c]);
                if (!v.empty())
                    RSG_CHECK_HIP(hipMemcpy(v.data(), H.scatter_items[c], sizeof(int2) * v.size(),
                                            hipMemcpyDeviceToHost));
                for (const int2 &e : v)
                    for (int ct = 0; ct < nct; ++ct) sitems[c].push_back(make_int4((int)i, e.x, e.y, ct));
            }
        }
    }
    // the stage outputs of all systems together decide the store policy
    double out_bytes = 0;
    for (const auto &d : b.sys) out_bytes += (double)d.nst * (double)d.ham->g->np * 16.0;
    b.nt = out_bytes >= kNtStoreBytes;
    int rc;
    for (int k = 0; k < 4; ++k) {
        if ((rc = upload(&b.sp[k], sp[k], s))) return rc;
        if ((rc = upload(&b.kb[k], kb[k], s))) return rc;
    }
    const std::vector<int32_t> ctr0(kBatchQueues + 1, 0);  // lives until the stream synchronisation below
    if ((rc = upload(&b.ctr, ctr0, s))) return rc;
    if ((rc = upload(&b.gitems, gitems, s))) return rc;
    if ((rc = upload(&b.sumitems, sumitems, s))) return rc;
    b.ngitems = (int32_t)gitems.size();
    b.nsumitems = (int32_t)sumitems.size();
    for (auto &v : sitems) {
        int4 *dptr = nullptr;
        if ((rc = upload(&dptr, v, s))) return rc;
        b.sitems.push_back(dptr);
        b.nsitems.push_back((int32_t)v.size());
    }
    RSG_CHECK_HIP(hipStreamSynchronize(s));
    for (size_t c = 0; c < b.cls.size(); ++c)
        if ((rc = build_class(b, c, s))) return rc;
    return RSG_OK;
}

int class_grid(const Batch &b, const BatchClass &c) {
    return b.grid_cap > 0 ? std::min(c.grid, (int)b.grid_cap) : c.grid;
}

// The persistent stencil launch of one class for stage k with factor (cre, cim).
int class_launch(const Batch &b, const BatchClass &c, int k, double cre, double cim, hipStream_t s) {
    return launch_stencil_batch(c.tile, 1, true, b.nt, b.sp[k], c.items, c.seg, c.nitems, cre, cim, b.ctr,
                                class_grid(b, c), s);
}

// Stage k of a step, the same product form as a single system's FP64 step:
// y <- y + (i dt / r_k) H y over the roots r_k of the Taylor(4) polynomial
// (every stage reads only its input; psi -> w1 -> w2 -> w1 -> psi).
int stage_launches(const Batch &b, int k, double dt, hipStream_t s) {
    const std::complex<double> c = std::complex<double>(0.0, dt) / taylor4_roots()[k];
    int rc;
    if ((rc = launch_kb_gather_batch(b.kb[k], b.gitems, b.ngitems, s))) return rc;
    if ((rc = launch_kb_gather_sum_batch(b.kb[k], b.sumitems, b.nsumitems, s))) return rc;
    // the classes' launches share the work counters: they run one after the
    // other on this stream, and each leaves the counters zero
    for (const auto &cl : b.cls)
        if ((rc = class_launch(b, cl, k, c.real(), c.imag(), s))) return rc;
    for (size_t ci = 0; ci < b.sitems.size(); ++ci)
        if ((rc = launch_kb_scatter_batch(b.kb[k], b.sitems[ci], b.nsitems[ci], c.real(), c.imag(), s)))
            return rc;
    return RSG_OK;
}

int steps(const Batch &b, double dt, int64_t nsteps, hipStream_t s) {
    for (int64_t n = 0; n < nsteps; ++n)
        for (int k = 0; k < 4; ++k) {
            const int rc = stage_launches(b, k, dt, s);
            if (rc) return rc;
        }
    return RSG_OK;
}

}  // namespace

}  // namespace rsg

using namespace rsg;

struct rsg_batch_s : rsg::Batch {};

static int check_systems(int32_t nsys, const rsg_system_desc *sys) {
    RSG_REQUIRE(nsys >= 1 && sys, RSG_EINVAL, "batch: need at least one system");
    for (int32_t i = 0; i < nsys; ++i) {
        const rsg_system_desc &d = sys[i];
        RSG_REQUIRE(d.ham, RSG_EINVAL, "batch: system %d has no Hamiltonian", i);
        RSG_REQUIRE(d.nst >= 1 && d.ldp >= 1 && d.ldp >= d.ham->g->np, RSG_ESHAPE,
                    "batch: system %d needs nst >= 1 and ldp >= np", i);
        RSG_REQUIRE(d.psi && ((uintptr_t)d.psi & 15) == 0, RSG_EINVAL, "batch: system %d orbital pointer", i);
        RSG_REQUIRE(d.ham->axis < 0, RSG_EUNSUPPORTED, "batch: system %d has a dipole field (not batched)", i);
        RSG_REQUIRE(!d.ham->mask, RSG_EUNSUPPORTED, "batch: system %d has an absorber mask (not batched)", i);
        RSG_REQUIRE(!d.ham->complex_scaled(), RSG_EUNSUPPORTED, "batch: system %d is complex-scaled (not batched)",
                    i);
        RSG_REQUIRE(d.ham->g->np < ((int64_t)1 << 27), RSG_EUNSUPPORTED, "batch: system %d has 2^27 points or more", i);
    }
    return RSG_OK;
}

extern "C" size_t rsg_batch_workspace_bytes(int32_t nsys, const rsg_system_desc *sys) {
    if (nsys < 1 || !sys) return 0;
    size_t n = 256;
    for (int32_t i = 0; i < nsys; ++i) {
        if (!sys[i].ham || sys[i].ldp < 1 || sys[i].nst < 0) return 0;
        n += sys_bytes(sys[i]);
    }
    return n;
}

// Systems -> size classes by tight-box width (kClassEdges), empty classes
// dropped; every class starts with the 32 x 8 depth-2 tile.
static void default_classes(Batch &b) {
    constexpr int ncl = (int)(sizeof(kClassEdges) / sizeof(kClassEdges[0])) + 1;
    std::vector<BatchClass> cls(ncl);
    for (size_t i = 0; i < b.sys.size(); ++i) {
        const int w = b.sys[i].ham->g->n[0];
        int c = 0;
        while (c < ncl - 1 && w >= kClassEdges[c]) ++c;
        cls[c].sys.push_back((int32_t)i);
    }
    b.cls.clear();
    for (auto &c : cls)
        if (!c.sys.empty()) {
            c.tile = TileShape{1, 32, 8, 0};
            c.tile.PD = 2;
            b.cls.push_back(c);
        }
}

static bool compiled_fp64(const rsg_tile *t) {
    for (const auto &c : tile_candidates(0))
        if (c.B == t->B && c.TX == t->TX && c.TY == t->TY && c.PD == t->PD) return true;
    return false;
}

extern "C" int rsg_batch_create(int32_t nsys, const rsg_system_desc *sys, void *ws, size_t ws_bytes,
                                void *stream, rsg_batch_t *out) {
    clear_error();
    int rc = check_systems(nsys, sys);
    if (rc) return rc;
    RSG_REQUIRE(out, RSG_EINVAL, "rsg_batch_create: null output");
    RSG_REQUIRE(ws && ws_bytes >= rsg_batch_workspace_bytes(nsys, sys), RSG_ENOMEM,
                "rsg_batch_create: workspace too small (%zu < %zu)", ws_bytes, rsg_batch_workspace_bytes(nsys, sys));
    return guarded([&]() -> int {
        hipStream_t s = (hipStream_t)stream;
        auto *b = new rsg_batch_s();
        b->sys.assign(sys, sys + nsys);
        char *base = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
        for (int32_t i = 0; i < nsys; ++i) {
            const size_t bb = rnd((size_t)sys[i].nst * (size_t)sys[i].ldp * 16);
            b->w1.push_back(base);
            b->w2.push_back(base + bb);
            b->D.push_back(base + 2 * bb);
            base += sys_bytes(sys[i]);
        }
        // zero the work buffers once, so timing runs never read garbage
        const hipError_t e = hipMemsetAsync(ws, 0, ws_bytes, s);
        if (e != hipSuccess) {
            set_error("rsg_batch_create: %s", hipGetErrorString(e));
            delete b;
            return RSG_EHIP;
        }
        default_classes(*b);
        const int r = build_tables(*b, s);
        if (r) {
            delete b;
            return r;
        }
        *out = b;
        return RSG_OK;
    });
}

extern "C" int rsg_batch_plan_create(int32_t nsys, const rsg_system_desc *sys, void *ws, size_t ws_bytes,
                                     void *stream, rsg_batch_t *out) {
    return rsg_batch_create(nsys, sys, ws, ws_bytes, stream, out);
}

extern "C" int rsg_batch_destroy(rsg_batch_t b) {
    clear_error();
    delete b;
    return RSG_OK;
}

extern "C" int rsg_batch_classes(rsg_batch_t b, int32_t *nclass, int32_t *class_of_sys) {
    clear_error();
    RSG_REQUIRE(b && nclass, RSG_EINVAL, "rsg_batch_classes: null argument");
    *nclass = (int32_t)b->cls.size();
    if (class_of_sys)
        for (size_t c = 0; c < b->cls.size(); ++c)
            for (const int32_t i : b->cls[c].sys) class_of_sys[i] = (int32_t)c;
    return RSG_OK;
}

extern "C" int rsg_batch_set_classes(rsg_batch_t b, const int32_t *class_of_sys, void *stream) {
    clear_error();
    RSG_REQUIRE(b && class_of_sys, RSG_EINVAL, "rsg_batch_set_classes: null argument");
    const int32_t nsys = (int32_t)b->sys.size();
    int32_t ncl = 0;
    for (int32_t i = 0; i < nsys; ++i) {
        RSG_REQUIRE(class_of_sys[i] >= 0 && class_of_sys[i] < nsys, RSG_EINVAL,
                    "rsg_batch_set_classes: class %d of system %d outside 0..nsys-1", class_of_sys[i], i);
        ncl = std::max(ncl, class_of_sys[i] + 1);
    }
    return guarded([&]() -> int {
        std::vector<BatchClass> cls(ncl);
        for (int32_t i = 0; i < nsys; ++i) cls[class_of_sys[i]].sys.push_back(i);
        for (int32_t c = 0; c < ncl; ++c)
            RSG_REQUIRE(!cls[c].sys.empty(), RSG_EINVAL, "rsg_batch_set_classes: class %d has no system", c);
        for (auto &c : cls) {
            c.tile = TileShape{1, 32, 8, 0};
            c.tile.PD = 2;
        }
        b->free_tables();
        b->cls = cls;
        return build_tables(*b, (hipStream_t)stream);
    });
}

static int set_class_tile(rsg_batch_t b, int32_t c, const rsg_tile *t) {
    BatchClass &cl = b->cls[c];
    cl.tile = TileShape{t->B, t->TX, t->TY, t->ZC};
    cl.tile.PD = t->PD;
    cl.tile.ZM = t->ZM;
    return RSG_OK;
}

static int check_batch_tile(const rsg_tile *t, const char *who) {
    RSG_REQUIRE(compiled_fp64(t), RSG_EUNSUPPORTED, "%s: not a compiled FP64 tile", who);
    RSG_REQUIRE(t->ZC >= 0, RSG_EINVAL, "%s: ZC must be >= 0", who);
    RSG_REQUIRE(t->ZM >= 0 && t->ZM <= 2, RSG_EINVAL, "%s: ZM must be 0, 1 or 2", who);
    return RSG_OK;
}

extern "C" int rsg_batch_set_tile(rsg_batch_t b, const rsg_tile *t, void *stream) {
    clear_error();
    RSG_REQUIRE(b && t, RSG_EINVAL, "rsg_batch_set_tile: null argument");
    int rc = check_batch_tile(t, "rsg_batch_set_tile");
    if (rc) return rc;
    return guarded([&]() -> int {
        for (int32_t c = 0; c < (int32_t)b->cls.size(); ++c) {
            set_class_tile(b, c, t);
            const int r = build_class(*b, (size_t)c, (hipStream_t)stream);
            if (r) return r;
        }
        return RSG_OK;
    });
}

extern "C" int rsg_batch_set_class_tile(rsg_batch_t b, int32_t c, const rsg_tile *t, void *stream) {
    clear_error();
    RSG_REQUIRE(b && t, RSG_EINVAL, "rsg_batch_set_class_tile: null argument");
    RSG_REQUIRE(c >= 0 && c < (int32_t)b->cls.size(), RSG_EINVAL, "rsg_batch_set_class_tile: no class %d", c);
    int rc = check_batch_tile(t, "rsg_batch_set_class_tile");
    if (rc) return rc;
    set_class_tile(b, c, t);
    return guarded([&]() { return build_class(*b, (size_t)c, (hipStream_t)stream); });
}

static rsg_tile tile_out(const TileShape &s) { return rsg_tile{s.B, s.TX, s.TY, s.ZC, s.PD, 0, 0, s.ZM}; }

extern "C" int rsg_batch_get_tile(rsg_batch_t b, rsg_tile *t) {
    clear_error();
    RSG_REQUIRE(b && t, RSG_EINVAL, "rsg_batch_get_tile: null argument");
    // the tile of the class with the most work
    size_t best = 0;
    int64_t bw = -1;
    for (size_t c = 0; c < b->cls.size(); ++c) {
        int64_t w = 0;
        for (const int32_t i : b->cls[c].sys) w += b->sys[i].ham->g->np * b->sys[i].nst;
        if (w > bw) {
            bw = w;
            best = c;
        }
    }
    *t = tile_out(b->cls[best].tile);
    return RSG_OK;
}

extern "C" int rsg_batch_get_class_tile(rsg_batch_t b, int32_t c, rsg_tile *t) {
    clear_error();
    RSG_REQUIRE(b && t, RSG_EINVAL, "rsg_batch_get_class_tile: null argument");
    RSG_REQUIRE(c >= 0 && c < (int32_t)b->cls.size(), RSG_EINVAL, "rsg_batch_get_class_tile: no class %d", c);
    *t = tile_out(b->cls[c].tile);
    return RSG_OK;
}

extern "C" int rsg_batch_class_info(rsg_batch_t b, int32_t c, int32_t *nsys, int64_t *nitems, int32_t *grid) {
    clear_error();
    RSG_REQUIRE(b, RSG_EINVAL, "rsg_batch_class_info: null batch");
    RSG_REQUIRE(c >= 0 && c < (int32_t)b->cls.size(), RSG_EINVAL, "rsg_batch_class_info: no class %d", c);
    const BatchClass &cl = b->cls[c];
    if (nsys) *nsys = (int32_t)cl.sys.size();
    if (nitems) *nitems = cl.nitems;
    if (grid) *grid = std::min<int64_t>(cl.nitems, class_grid(*b, cl));
    return RSG_OK;
}

extern "C" int rsg_batch_set_grid(rsg_batch_t b, int32_t max_workgroups) {
    clear_error();
    RSG_REQUIRE(b, RSG_EINVAL, "rsg_batch_set_grid: null batch");
    RSG_REQUIRE(max_workgroups >= 0, RSG_EINVAL, "rsg_batch_set_grid: max_workgroups must be >= 0");
    b->grid_cap = max_workgroups;
    b->drop_graphs();  // captured launches hold the old grid size
    return RSG_OK;
}

// Per class: every compiled tile x z-chunk {whole, 32} x z-march {upward,
// centre-out}, timed on that class's persistent launch of a middle stage
// (w1 -> w2, the orbitals untouched), best of reps after a warm-up; the
// fastest per class is kept.
extern "C" int rsg_batch_autotune(rsg_batch_t b, int32_t reps, rsg_tile *best, double *best_ms, void *stream) {
    clear_error();
    RSG_REQUIRE(b && reps > 0, RSG_EINVAL, "rsg_batch_autotune: bad argument");
    hipStream_t s = (hipStream_t)stream;
    return guarded([&]() -> int {
        hipEvent_t e0, e1;
        RSG_CHECK_HIP(hipEventCreate(&e0));
        RSG_CHECK_HIP(hipEventCreate(&e1));
        int rc = RSG_OK;
        double total = 0.0;
        std::vector<TileShape> chosen;
        for (auto &c : b->cls) chosen.push_back(c.tile);
        for (size_t ci = 0; ci < b->cls.size() && !rc; ++ci) {
            double bt = 1e300;
            for (const auto &cand : tile_candidates(0)) {
                for (int zv = 0; zv < 4; ++zv) {
                    TileShape sh = cand;
                    sh.ZC = (zv & 1) ? 32 : 0;
                    sh.ZM = zv >> 1;
                    b->cls[ci].tile = sh;
                    if ((rc = build_class(*b, ci, s))) break;
                    double tmin = 1e300;
                    for (int r = 0; r <= reps; ++r) {
                        RSG_CHECK_HIP(hipEventRecord(e0, s));
                        if ((rc = class_launch(*b, b->cls[ci], 1, 0.0, -1e-3, s))) break;
                        RSG_CHECK_HIP(hipEventRecord(e1, s));
                        RSG_CHECK_HIP(hipEventSynchronize(e1));
                        float ms = 0.f;
                        RSG_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
                        if (r > 0) tmin = std::min(tmin, (double)ms);
                    }
                    if (rc) break;
                    if (tmin < bt) {
                        bt = tmin;
                        chosen[ci] = sh;
                    }
                }
                if (rc) break;
            }
            b->cls[ci].tile = chosen[ci];
            total += bt;
            if (!rc) rc = build_class(*b, ci, s);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) {
            // leave a consistent batch behind: every class on its chosen tile
            for (size_t ci = 0; ci < b->cls.size(); ++ci) b->cls[ci].tile = chosen[ci];
            (void)build_tables(*b, s);
            return rc;
        }
        if (best) rsg_batch_get_tile(b, best);
        if (best_ms) *best_ms = total;
        return RSG_OK;
    });
}

extern "C" int rsg_batch_propagate(rsg_batch_t b, double dt, int64_t nsteps, int32_t use_graph, void *stream) {
    clear_error();
    RSG_REQUIRE(b, RSG_EINVAL, "rsg_batch_propagate: null batch");
    RSG_REQUIRE(nsteps >= 0 && std::isfinite(dt), RSG_EINVAL, "rsg_batch_propagate: bad nsteps or dt");
    hipStream_t s = (hipStream_t)stream;
    if (nsteps == 0) return RSG_OK;
    if (!use_graph) return steps(*b, dt, nsteps, s);
    RSG_REQUIRE(s != nullptr, RSG_EINVAL, "rsg_batch_propagate: graph capture needs a non-default stream");
    const auto key = std::make_tuple(dt, nsteps, s);
    auto it = b->graphs.find(key);
    hipGraphExec_t exec = it == b->graphs.end() ? nullptr : it->second;
    if (!exec) {
        RSG_CHECK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const int r = steps(*b, dt, nsteps, s);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &graph);
        if (r) {
            if (graph) (void)hipGraphDestroy(graph);
            return r;
        }
        if (e != hipSuccess) {
            set_error("rsg_batch_propagate: capture failed: %s", hipGetErrorString(e));
            return RSG_EHIP;
        }
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            set_error("rsg_batch_propagate: instantiate failed: %s", hipGetErrorString(ei));
            return RSG_EHIP;
        }
        b->graphs[key] = exec;
    }
    RSG_CHECK_HIP(hipGraphLaunch(exec, s));
    return RSG_OK;
}

extern "C" int rsg_batch_run(rsg_batch_t b, int64_t nsteps, double dt, void *stream) {
    return rsg_batch_propagate(b, dt, nsteps, 1, stream);
}
