// Host side of libbxmg: BoxArrays, MultiFabs, cached ghost-copy plans, the
// multigrid hierarchy and the V-cycle driver, behind the C ABI of bxmg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <array>
#include <atomic>
#include <stdexcept>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/bxmg.h"
#include "bxmg_internal.h"
#include "bxmg_host.h"

thread_local std::string g_err;
std::atomic<uint64_t> g_next_id{1};

// ================================================================ hierarchy
namespace {

template <class T>
struct FaceSet {
    DevBuf<T> c[3];
    DevBuf<FaceArrays<T>> table;  // one entry (problem slot 0): the view below
    FaceArrays<T> view(const Box& dom) const {
        FaceArrays<T> f;
        for (int d = 0; d < 3; ++d) { f.c[d] = c[d].p; f.dlo[d] = dom.lo[d]; f.n[d] = dom.n(d); }
        return f;
    }
};

template <class T>
FaceArrays<T> no_faces() {
    FaceArrays<T> f;
    for (int d = 0; d < 3; ++d) { f.c[d] = nullptr; f.dlo[d] = 0; f.n[d] = 0; }
    return f;
}

struct GhostList {
    DevBuf<GhostCopy> list;
    long long n = 0;
    void set(const std::vector<GhostCopy>& v) {
        list.upload(v);
        n = (long long)v.size();
    }
};

struct Level {
    Box dom;
    double h;
    std::vector<Box> boxes;
    std::vector<RBox> rb;
    DevBuf<RBox> d_rb;
    long long nelem = 0;
    // colour-cell tiles (valid cells, one colour per thread per plane)
    DevBuf<Tile> tcol;
    int ntcol = 0;
    // transfer tiles to level + 1 (coarse cells of every box)
    DevBuf<Tile> tdown;
    int ntdown = 0;
    DevBuf<int> cbox;
    // coefficient setup tiles (coarse faces anchored in every box), level 0
    DevBuf<Tile> tface[3];
    int ntface[3] = {0, 0, 0};
    GhostList face[2];  // face ghosts of colour c: exchange + Dirichlet
    GhostList full;     // every ghost: exchange + Dirichlet
    GhostList full_even;  // every ghost: exchange + even reflection (cell beta)
    bool push = false;    // producers refresh the face ghosts they mirror
    mutable int flip = 0; // direction of the next sweep over the level's tiles
    bool res = false;     // 32-bit buffer addressing of the boxes
    // level 0 of a solve whose caller boxes were merged: one view per caller
    // box (its valid cells, addressed in the merged storage) and tiles over
    // them, for the layout conversions and the field norm
    bool merged = false;
    DevBuf<RBox> d_vrb;
    DevBuf<Tile> tview;
    int ntview = 0;
    Grid view_grid() const { return merged ? Grid{d_vrb.p, tview.p, ntview, 0, nullptr, 0, 0} : grid(); }
    // level 0: the fixed tiles of the periodic mean (mean_tiles over the
    // caller's boxes, so the sum's order does not depend on merging)
    DevBuf<Tile> tmean;
    int ntmean = 0;
    Grid mean_grid() const {
        return merged ? Grid{d_vrb.p, tmean.p, ntmean, 0, nullptr, 0, 0}
                      : Grid{d_rb.p, tmean.p, ntmean, push ? 1 : 0, nullptr, 0, res ? 1 : 0};
    }
    int stage_values = 0;  // coarse values a colour tile reads in a prolongation (bound)
    Grid grid() const { return Grid{d_rb.p, tcol.p, ntcol, push ? (boxes.size() == 1 ? 2 : 1) : 0, nullptr, 0, res ? 1 : 0}; }
    // grid of the next sweep in the alternating order (see tile_index)
    Grid walk() const {
        Grid g = grid();
        g.rev = flip;
        flip ^= 1;
        return g;
    }

};

}  // namespace

struct Hier {
    int per[3];
    int precision;
    bool var;
    double alpha = 0.0;  // Helmholtz coefficient of every level's operator
    std::vector<std::unique_ptr<Level>> L;
    // FP64 storage: all levels (precision 0) or level 0 only (precision 1)
    std::vector<std::unique_ptr<DevBuf<double>>> u64, f64;
    std::vector<std::unique_ptr<DevBuf<float>>> u32, f32;
    DevBuf<double> beta64;
    DevBuf<float> beta32;
    std::vector<std::unique_ptr<FaceSet<double>>> faces64;  // index = level (0 unused)
    std::vector<std::unique_ptr<FaceSet<float>>> faces32;
    int coarse_start = -1;    // first level of the fused coarse cycle (-1: none)
    DevBuf<CoarseCycle<double>> cc64;  // device copies of the descriptors ...
    DevBuf<CoarseCycle<float>> cc32;
    CoarseCycle<double> cc64_host{};   // ... and what they hold
    CoarseCycle<float> cc32_host{};
    int cc64_lds = 0, cc32_lds = 0;    // dynamic LDS of the coarse-cycle launch
    DevBuf<double> partials;  // 3 per tile of the largest tiled launch, + 3
    DevBuf<double> fnorm;     // 3
    // the solve's stop test on the device (the batch engine's, one slot):
    // slot state, flags {active, slot index 0, active count, guess not +0}, the history
    // (kHist of |r|/|f|, then kHist of |r|_2) and the norms of f
    DevBuf<BatchSlot> st;
    DevBuf<int> flags;
    DevBuf<double> hist;
    DevBuf<double> fn3;
    DevBuf<int> iters;
    // multigrid-preconditioned CG on level 0 (allocated by its first solve):
    // residual, two directions (read one, write the other), q = L p, the
    // iterate and right-hand side when the FP64 V-cycle needs level 0's own
    // arrays, per-tile partial sums, their reduction and the scalars
    struct Krylov {
        DevBuf<double> r, q, x, f, part, sums;
        DevBuf<double> p[2];
        DevBuf<KrylovScalars> sc;
    } kr;
    size_t bytes = 0;
    XGrid xgrid(size_t l) const {
        const Level& F = *L[l];
        const Level& C = *L[l + 1];
        return XGrid{F.d_rb.p, C.d_rb.p, F.cbox.p, F.tdown.p, F.ntdown, F.push ? 1 : 0, nullptr, 0,
                     (F.res && C.res) ? 1 : 0};
    }
    XGrid xwalk(size_t l) const {
        XGrid x = xgrid(l);
        x.rev = L[l]->flip;
        L[l]->flip ^= 1;
        return x;
    }
    XGrid face_grid(int d) const {
        const Level& F = *L[0];
        const Level& C = *L[1];
        return XGrid{F.d_rb.p, C.d_rb.p, F.cbox.p, F.tface[d].p, F.ntface[d], 0, nullptr, 0, 0};
    }
};

// Tile depth: planes walked per thread in the cell kernels (a tuning knob,
// bxmg_ctx_tune), separately for tiles that span whole box planes.
struct Tuning {
    int zc = 4;
    int zc_planes = 4;
    int res = 1;
    int ly_cap = 8;
};

static void upload_tiles(const TileSet& t, DevBuf<Tile>& buf, int& n) {
    buf.upload(t.tiles);
    n = (int)t.tiles.size();
}

// merge: coarse levels run on execution_boxes (solves); the stage calls keep
// the logical boxes, which their caller's MultiFabs are laid out on.
static std::unique_ptr<Hier> build_hier(const bxmg_ba_s* ba, int precision, bool var, double h0, const Tuning& tune,
                                        bool merge, double alpha) {
    auto H = std::make_unique<Hier>();
    for (int d = 0; d < 3; ++d) H->per[d] = ba->per[d];
    H->precision = precision;
    H->var = var;
    H->alpha = alpha;
    std::vector<LevelBoxes> lb = make_hierarchy(ba->dom, ba->boxes);
    double h = h0;
    long long max_tiles = 1;
    for (size_t l = 0; l < lb.size(); ++l) {
        auto lv = std::make_unique<Level>();
        lv->dom = lb[l].dom;
        lv->h = h;
        h *= 2.0;
        lv->boxes = merge ? execution_boxes(lb[l], l, true) : lb[l].boxes;
        lv->rb = rb_layout(lv->boxes, 1, lv->h, &lv->nelem);
        for (auto& r : lv->rb) r.a = alpha;
        if (l == 0 && lv->boxes.size() != lb[0].boxes.size()) {
            // views of the caller's boxes: their own valid range, the merged
            // box's addressing (colour parity is global, so rb_idx and
            // colour_i agree with the merged box)
            lv->merged = true;
            std::vector<RBox> v;
            for (const Box& b : lb[0].boxes) {
                RBox r = lv->rb[0];
                for (int d = 0; d < 3; ++d) { r.lo[d] = b.lo[d]; r.hi[d] = b.hi[d]; }
                for (int q = 0; q < 6; ++q) { r.nb[q] = -1; r.shift[q] = 0; }
                v.push_back(r);
            }
            lv->d_vrb.upload(v);
            const TileSet tv =
                level_tiles(colour_extents(lb[0].boxes), tune.zc, tune.zc_planes, tune.ly_cap, kMinLevelTiles);
            upload_tiles(tv, lv->tview, lv->ntview);
            max_tiles = std::max<long long>(max_tiles, lv->ntview);
        }
        lv->push = face_neighbours(lv->dom, H->per, lv->boxes, lv->rb);
        lv->res = tune.res && boxes_fit_res(lv->rb);
        lv->d_rb.upload(lv->rb);
        {
            const TileSet ts =
                level_tiles(colour_extents(lv->boxes), tune.zc, tune.zc_planes, tune.ly_cap, kMinLevelTiles);
            upload_tiles(ts, lv->tcol, lv->ntcol);
            lv->stage_values = prolong_stage_values(ts.sh);
            if (l == 0) {
                upload_tiles(mean_tiles(colour_extents(lb[0].boxes)), lv->tmean, lv->ntmean);
                max_tiles = std::max<long long>(max_tiles, lv->ntmean);
            }
        }
        max_tiles = std::max<long long>(max_tiles, lv->ntcol);
        if (l + 1 < lb.size()) {
            upload_tiles(make_tiles(coarse_extents(lv->boxes, lv->dom, -1), tune.zc, tune.ly_cap, kMinLevelTiles),
                         lv->tdown, lv->ntdown);
            lv->cbox.upload(coarse_owner(lv->boxes, merge ? execution_boxes(lb[l + 1], l + 1) : lb[l + 1].boxes));
            if (var && l == 0)
                for (int d = 0; d < 3; ++d)
                    upload_tiles(make_tiles(coarse_extents(lv->boxes, lv->dom, d), tune.zc), lv->tface[d], lv->ntface[d]);
        }
        const std::vector<Tag> faces = build_tags(lv->dom, H->per, lv->boxes, 1, true, 2, true);
        lv->face[0].set(ghost_list(faces, lv->rb, 1));
        lv->face[1].set(ghost_list(faces, lv->rb, 2));
        lv->full.set(ghost_list(build_tags(lv->dom, H->per, lv->boxes, 1, false, 2, true), lv->rb, 3));
        if (l == 0 && var) lv->full_even.set(ghost_list(build_tags(lv->dom, H->per, lv->boxes, 1, false, 2, false), lv->rb, 3));
        H->L.push_back(std::move(lv));
    }
    const size_t nl = H->L.size();
    H->u64.resize(nl);
    H->f64.resize(nl);
    H->u32.resize(nl);
    H->f32.resize(nl);
    for (size_t l = 0; l < nl; ++l) {
        const long long n = H->L[l]->nelem;
        if (precision == 0 || l == 0) {
            H->u64[l] = std::make_unique<DevBuf<double>>();
            H->f64[l] = std::make_unique<DevBuf<double>>();
            H->u64[l]->alloc(n);
            H->f64[l]->alloc(n);
            HIPCHK(hipMemset(H->u64[l]->p, 0, n * 8));
            HIPCHK(hipMemset(H->f64[l]->p, 0, n * 8));
            H->bytes += 16 * n;
        }
        if (precision == 1) {
            H->u32[l] = std::make_unique<DevBuf<float>>();
            H->f32[l] = std::make_unique<DevBuf<float>>();
            H->u32[l]->alloc(n);
            H->f32[l]->alloc(n);
            HIPCHK(hipMemset(H->u32[l]->p, 0, n * 4));
            HIPCHK(hipMemset(H->f32[l]->p, 0, n * 4));
            H->bytes += 8 * n;
        }
    }
    if (var) {
        H->beta64.alloc(H->L[0]->nelem);
        HIPCHK(hipMemset(H->beta64.p, 0, H->L[0]->nelem * 8));
        if (precision == 1) {
            H->beta32.alloc(H->L[0]->nelem);
            HIPCHK(hipMemset(H->beta32.p, 0, H->L[0]->nelem * 4));
        }
        H->faces64.resize(nl);
        H->faces32.resize(nl);
        for (size_t l = 1; l < nl; ++l) {
            const Box& D = H->L[l]->dom;
            for (int d = 0; d < 3; ++d) {
                const size_t nf = (size_t)(D.n(0) + (d == 0)) * (D.n(1) + (d == 1)) * (D.n(2) + (d == 2));
                if (precision == 0) {
                    if (!H->faces64[l]) H->faces64[l] = std::make_unique<FaceSet<double>>();
                    H->faces64[l]->c[d].alloc(nf);
                } else {
                    if (!H->faces32[l]) H->faces32[l] = std::make_unique<FaceSet<float>>();
                    H->faces32[l]->c[d].alloc(nf);
                }
            }
            if (precision == 0) H->faces64[l]->table.upload({H->faces64[l]->view(D)});
            else H->faces32[l]->table.upload({H->faces32[l]->view(D)});
        }
    }
    H->partials.alloc(6 * max_tiles + 8);  // two sets: the fused residual's colour-1 and colour-0 norms
    H->fnorm.alloc(4);
    H->st.alloc(1);
    H->flags.alloc(4);
    HIPCHK(hipMemset(H->flags.p, 0, 4 * sizeof(int)));
    H->hist.alloc(2 * kHist);
    H->fn3.alloc(4);
    H->iters.alloc(1);
    // fused coarse cycle: from the first level l >= 1 below which every level
    // is one box of at most kMaxBottomCells cells
    for (size_t l = 1; l < nl; ++l) {
        bool ok = nl - l <= (size_t)kMaxCoarseLevels;
        for (size_t m = l; m < nl && ok; ++m)
            ok = H->L[m]->boxes.size() == 1 && H->L[m]->dom.cells() <= kMaxBottomCells;
        if (ok) { H->coarse_start = (int)l; break; }
    }
    return H;
}

// Device descriptor of the fused coarse cycle for storage type T.
template <class T>
static CoarseCycle<T> coarse_desc(Hier* H, int nu1, int nu2, int prolong, double rtol);

// ================================================================== driver
namespace {

template <class T>
T* lvl_u(Hier* H, size_t l);
template <>
double* lvl_u<double>(Hier* H, size_t l) { return H->u64[l]->p; }
template <>
float* lvl_u<float>(Hier* H, size_t l) { return H->u32[l]->p; }
template <class T>
T* lvl_f(Hier* H, size_t l);
template <>
double* lvl_f<double>(Hier* H, size_t l) { return H->f64[l]->p; }
template <>
float* lvl_f<float>(Hier* H, size_t l) { return H->f32[l]->p; }

template <class T>
const T* lvl_beta(Hier* H, size_t l);
template <>
const double* lvl_beta<double>(Hier* H, size_t l) { return (H->var && l == 0) ? H->beta64.p : nullptr; }
template <>
const float* lvl_beta<float>(Hier* H, size_t l) { return (H->var && l == 0) ? H->beta32.p : nullptr; }

template <class T>
FaceArrays<T> lvl_faces(Hier* H, size_t l);
template <>
FaceArrays<double> lvl_faces<double>(Hier* H, size_t l) {
    if (!H->var || l == 0) return no_faces<double>();
    return H->faces64[l]->view(H->L[l]->dom);
}
template <>
FaceArrays<float> lvl_faces<float>(Hier* H, size_t l) {
    if (!H->var || l == 0) return no_faces<float>();
    return H->faces32[l]->view(H->L[l]->dom);
}

// device table of the level's face arrays (MODE 2 stencils), or nullptr
template <class T>
const FaceArrays<T>* lvl_fat(Hier* H, size_t l);
template <>
const FaceArrays<double>* lvl_fat<double>(Hier* H, size_t l) {
    return (!H->var || l == 0) ? nullptr : H->faces64[l]->table.p;
}
template <>
const FaceArrays<float>* lvl_fat<float>(Hier* H, size_t l) {
    return (!H->var || l == 0) ? nullptr : H->faces32[l]->table.p;
}

}  // namespace

template <class T>
static CoarseCycle<T> coarse_desc(Hier* H, int nu1, int nu2, int prolong, double rtol) {
    CoarseCycle<T> cc;
    std::memset(&cc, 0, sizeof cc);
    const size_t l0 = (size_t)H->coarse_start;
    cc.nlev = (int)(H->L.size() - l0);
    cc.nu1 = nu1;
    cc.nu2 = nu2;
    cc.prolong = prolong;
    for (int d = 0; d < 3; ++d) cc.per[d] = H->per[d];
    cc.rtol = rtol;
    cc.iters = H->iters.p;
    for (int m = 0; m < cc.nlev; ++m) {
        const Level& L = *H->L[l0 + m];
        CoarseLevel<T>& c = cc.L[m];
        c.box = L.rb[0];
        c.u = lvl_u<T>(H, l0 + m);
        c.f = lvl_f<T>(H, l0 + m);
        for (int q = 0; q < 2; ++q) { c.face[q] = L.face[q].list.p; c.nface[q] = L.face[q].n; }
        c.full = L.full.list.p;
        c.nfull = L.full.n;
        c.nelem = L.nelem;
        c.h = L.h;
        c.fa = lvl_faces<T>(H, l0 + m);
        c.push = L.push ? 1 : 0;
    }
    return cc;
}

namespace {

struct Run {
    Hier* H;
    hipStream_t s;
    int nu1, nu2, prolong;
    double bottom_rtol;
    Profiler* prof = nullptr;
    bool lds_coarse = true;  // the fused coarse cycle may keep its levels in LDS
    // the solve's stop flag (active[0]); the V-cycle's kernels do nothing
    // once the device-side stop test has cleared it
    const int* active = nullptr;
    // fused residual: the last level-0 colour-1 sweep of the V-cycle writes
    // its cells' residual norms here (and sets fused_sweep), so the stop test
    // needs the colour-0 residual only
    double* fuse_norms = nullptr;
    bool fused_sweep = false;
    Grid grid(const Grid& g) const {
        Grid r = g;
        r.active = active;
        return r;
    }
    // event brackets around level-0 launches of the profiled stage
    void pre(size_t l, int stage) { if (prof && prof->stage == stage && l == 0) prof->mark(s); }
    void post(size_t l, int stage) { if (prof && prof->stage == stage && l == 0) prof->mark(s); }
};

enum { kStageGS = 0, kStageResid = 1, kStageRestrict = 2, kStageProlong = 3, kStageFill = 4, kStageCoarse = 5 };

template <class T>
void fill(Run& R, size_t l, T* data, const GhostList& g) {
    R.pre(l, kStageFill);
    HIPCHK(launch_fill_rb(R.s, data, sizeof(T) == 4, g.list.p, g.n, R.active));
    R.post(l, kStageFill);
}

// both colours' face ghosts: two lists (the solver refreshes them per colour)
template <class T>
void fill_faces(Run& R, size_t l, T* data) {
    const Level& L = *R.H->L[l];
    fill<T>(R, l, data, L.face[0]);
    fill<T>(R, l, data, L.face[1]);
}

// post: the post-smoothing, whose last level-0 sweep may carry the fused
// residual norms
template <class T>
void smooth(Run& R, size_t l, int nsweeps, bool post = false) {
    Hier* H = R.H;
    const Level& L = *H->L[l];
    T* u = lvl_u<T>(H, l);
    const T* f = lvl_f<T>(H, l);
    for (int s = 0; s < nsweeps; ++s)
        for (int c = 0; c < 2; ++c) {
            if (!L.push) fill<T>(R, l, u, L.face[c ^ 1]);
            const bool fuse = R.fuse_norms && l == 0 && post && s == nsweeps - 1 && c == 1;
            R.pre(l, kStageGS);
            HIPCHK(launch_gs<T>(R.s, R.grid(L.walk()), u, f, lvl_beta<T>(H, l), lvl_fat<T>(H, l), c,
                                fuse ? R.fuse_norms : nullptr));
            R.post(l, kStageGS);
            if (fuse) R.fused_sweep = true;
        }
}

template <class T>
void bottom(Run& R, size_t l) {
    Hier* H = R.H;
    const Level& L = *H->L[l];
    HIPCHK(launch_bottom<T>(R.s, lvl_u<T>(H, l), lvl_f<T>(H, l), lvl_faces<T>(H, l), H->var && l > 0, L.d_rb.p,
                            (int)L.boxes.size(), L.dom.lo, L.dom.hi, H->per, L.h, H->alpha, R.bottom_rtol, H->iters.p));
}

template <class T>
DevBuf<CoarseCycle<T>>& cc_buf(Hier* H);
template <>
DevBuf<CoarseCycle<double>>& cc_buf<double>(Hier* H) { return H->cc64; }
template <>
DevBuf<CoarseCycle<float>>& cc_buf<float>(Hier* H) { return H->cc32; }
template <class T>
CoarseCycle<T>& cc_host(Hier* H);
template <>
CoarseCycle<double>& cc_host<double>(Hier* H) { return H->cc64_host; }
template <>
CoarseCycle<float>& cc_host<float>(Hier* H) { return H->cc32_host; }

// the fused coarse cycle; its descriptor is uploaded when the settings change
template <class T>
int& cc_lds(Hier* H);
template <>
int& cc_lds<double>(Hier* H) { return H->cc64_lds; }
template <>
int& cc_lds<float>(Hier* H) { return H->cc32_lds; }

template <class T>
void coarse_cycle(Run& R) {
    Hier* H = R.H;
    static_assert(std::is_trivially_copyable<CoarseCycle<T>>::value, "descriptor must be plain data");
    DevBuf<CoarseCycle<T>>& buf = cc_buf<T>(H);
    CoarseCycle<T>& host = cc_host<T>(H);
    CoarseCycle<T> cc = coarse_desc<T>(H, R.nu1, R.nu2, R.prolong, R.bottom_rtol);
    const int lds = coarse_lds_layout<T>(cc, R.lds_coarse);
    if (!buf.p || std::memcmp(&cc, &host, sizeof cc) != 0) {
        if (!buf.p) buf.alloc(1);
        host = cc;  // lives as long as the hierarchy: safe source for the async copy
        cc_lds<T>(H) = lds;
        HIPCHK(hipMemcpyAsync(buf.p, &host, sizeof host, hipMemcpyHostToDevice, R.s));
    }
    // (the kernel zeroes the top level's correction itself)
    HIPCHK(launch_coarse_cycle<T>(R.s, buf.p, 1, R.active, H->var, cc_lds<T>(H), host.lds != 0));
}

template <class T>
void vcycle(Run& R, size_t l) {
    Hier* H = R.H;
    const size_t last = H->L.size() - 1;
    if ((int)l == H->coarse_start) {
        R.pre(0, kStageCoarse);
        coarse_cycle<T>(R);
        R.post(0, kStageCoarse);
        return;
    }
    if (l == last) {
        bottom<T>(R, l);
        return;
    }
    const Level& L = *H->L[l];
    const Level& C = *H->L[l + 1];
    T* u = lvl_u<T>(H, l);
    smooth<T>(R, l, R.nu1);
    if (!L.push) fill_faces<T>(R, l, u);
    R.pre(l, kStageRestrict);
    XGrid x = H->xwalk(l);
    x.active = R.active;
    // the coarse correction starts from zero: zeroed by the same launch (the
    // fused coarse cycle zeroes its top level itself)
    const bool zero_c = (int)l + 1 != H->coarse_start;
    HIPCHK(launch_resid_restrict<T>(R.s, x, u, lvl_f<T>(H, l), lvl_beta<T>(H, l), lvl_fat<T>(H, l),
                                    lvl_f<T>(H, l + 1), zero_c ? lvl_u<T>(H, l + 1) : nullptr));
    R.post(l, kStageRestrict);
    vcycle<T>(R, l + 1);
    // a small one-box coarse level needs no ghost refresh where the staged
    // prolongation reads the cells its ghosts mirror (on large levels the
    // refresh launch costs less than the mirroring in every tile)
    const bool self = C.boxes.size() == 1 && C.dom.cells() <= kSelfGhostCells &&
                      prolong_staged(L.push, R.nu2 > 0, L.stage_values);
    if (!self) fill<T>(R, l + 1, lvl_u<T>(H, l + 1), C.full);
    R.pre(l, kStageProlong);
    // with post-smoothing, its first (colour-0) sweep overwrites colour 0
    // a large one-box fine level takes its face work in a second launch
    long long faces = 0;
    if (L.boxes.size() == 1 && !self) {
        const Box& b = L.boxes[0];
        faces = 2 * ((long long)b.n(1) * b.n(2) + (long long)b.n(0) * b.n(2) + (long long)b.n(0) * b.n(1));
    }
    HIPCHK(launch_prolong<T>(R.s, R.grid(L.walk()), C.d_rb.p, L.cbox.p, lvl_u<T>(H, l + 1), u, R.prolong, R.nu2 > 0,
                             L.stage_values, self, faces));
    R.post(l, kStageProlong);
    smooth<T>(R, l, R.nu2, true);
}

// Coefficient setup: cell beta at level 0 (exchange + even reflection), then
// face arrays level by level.
template <class T>
void setup_faces(Run& R, T* beta0) {
    Hier* H = R.H;
    const Level& L0 = *H->L[0];
    fill<T>(R, 0, beta0, L0.full_even);
    for (size_t l = 1; l < H->L.size(); ++l) {
        FaceArrays<T> out = lvl_faces<T>(H, l);
        for (int d = 0; d < 3; ++d) {
            T* dst = const_cast<T*>(out.c[d]);
            if (l == 1) HIPCHK(launch_faces_from_cells<T>(R.s, H->face_grid(d), beta0, d, out, dst));
            else HIPCHK(launch_faces_coarsen<T>(R.s, lvl_faces<T>(H, l - 1), out, d, dst));
        }
    }
}

// Host copy of a solve's stop-test state: the two histories, the slot, the flag.
struct SolveState {
    double hist[kHist];
    double hist_l2[kHist];
    BatchSlot st;
    int active;
};

double norm_readback(Run& R, double* h_norm, const double* dev) {
    HIPCHK(hipMemcpyAsync(h_norm, dev, 3 * sizeof(double), hipMemcpyDeviceToHost, R.s));
    HIPCHK(hipStreamSynchronize(R.s));
    return h_norm[0];
}

}  // namespace

// ================================================================== C ABI
// Host scatter/gather of one component between a domain-sized F-order host
// array and the valid cells of every box, through a host copy of the slab.
template <class T>
static void copy_valid(bxmg_multifab mf, std::vector<unsigned char>& slab, T* glob, int comp, bool to_dev) {
    T* sl = (T*)slab.data();
    const Box& D = mf->ba->dom;
    const long long nx = D.n(0), ny = D.n(1);
    for (size_t b = 0; b < mf->fboxes.size(); ++b) {
        const FBox& f = mf->fboxes[b];
        for (int k = f.lo[2]; k <= f.hi[2]; ++k)
            for (int j = f.lo[1]; j <= f.hi[1]; ++j) {
                T* row = sl + f.base + comp * f.cs +
                         (long long)(f.lo[0] - f.glo[0]) +
                         (long long)f.G[0] * ((long long)(j - f.glo[1]) + (long long)f.G[1] * (k - f.glo[2]));
                T* g = glob + (long long)(f.lo[0] - D.lo[0]) + nx * ((long long)(j - D.lo[1]) + ny * (k - D.lo[2]));
                const int n = f.hi[0] - f.lo[0] + 1;
                if (to_dev) std::memcpy(row, g, n * sizeof(T));
                else std::memcpy(g, row, n * sizeof(T));
            }
    }
}

extern "C" {

int bxmg_version(void) { return 100; }

const char* bxmg_last_error(void) { return g_err.c_str(); }

bxmg_status bxmg_ctx_create(int device, void* hip_stream, bxmg_ctx* out) {
    if (!out) return fail(BXMG_EINVAL, "ctx_create: out is NULL");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
        return fail(BXMG_EDEVICE, "ctx_create: no such HIP device");
    if (hipSetDevice(device) != hipSuccess) return fail(BXMG_EDEVICE, "ctx_create: hipSetDevice failed");
    auto* c = new bxmg_ctx_s();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    const hipError_t se = scratch_address(device, &c->scratch);  // with the device current
    if (se != hipSuccess) {
        delete c;
        return fail(BXMG_EDEVICE, std::string("ctx_create: staging array address: ") + hipGetErrorString(se));
    }
    if (hipHostMalloc((void**)&c->h_norm, 8 * sizeof(double)) != hipSuccess ||
        hipHostMalloc(&c->h_solve, sizeof(SolveState)) != hipSuccess) {
        if (c->h_norm) (void)hipHostFree(c->h_norm);
        delete c;
        return fail(BXMG_ENOMEM, "ctx_create: pinned host allocation failed");
    }
    *out = c;
    return BXMG_OK;
}

void bxmg_ctx_destroy(bxmg_ctx ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->cache.clear();
    ctx->composite.reset();
    ctx->nodal.reset();
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->h_norm) (void)hipHostFree(ctx->h_norm);
    if (ctx->h_solve) (void)hipHostFree(ctx->h_solve);
    delete ctx;
}

static bool valid_dom(const int32_t* lo, const int32_t* hi) {
    return lo && hi && lo[0] <= hi[0] && lo[1] <= hi[1] && lo[2] <= hi[2];
}

static bxmg_status make_ba(const int32_t* dom_lo, const int32_t* dom_hi, const int32_t* bc, std::vector<Box> boxes,
                           bxmg_boxarray* out) {
    auto* ba = new bxmg_ba_s();
    for (int d = 0; d < 3; ++d) {
        ba->dom.lo[d] = dom_lo[d];
        ba->dom.hi[d] = dom_hi[d];
        ba->bc[d] = bc ? bc[d] : BXMG_DIRICHLET0;
        ba->per[d] = (ba->bc[d] == BXMG_PERIODIC) ? 1 : 0;
    }
    ba->boxes = std::move(boxes);
    ba->id = g_next_id++;
    *out = ba;
    return BXMG_OK;
}

bxmg_status bxmg_define_boxarray(const int32_t dom_lo[3], const int32_t dom_hi[3], const int32_t bc[3],
                                 int32_t max_box_size, bxmg_boxarray* out) {
    if (!out || !valid_dom(dom_lo, dom_hi)) return fail(BXMG_EINVAL, "define_boxarray: empty domain");
    if (max_box_size < 1) return fail(BXMG_EINVAL, "define_boxarray: max_box_size < 1");
    for (int d = 0; d < 3; ++d)
        if (bc && bc[d] != BXMG_PERIODIC && bc[d] != BXMG_DIRICHLET0) return fail(BXMG_EINVAL, "define_boxarray: bad bc");
    std::vector<std::pair<int, int>> p[3];
    for (int d = 0; d < 3; ++d) p[d] = chop1(dom_lo[d], dom_hi[d] - dom_lo[d] + 1, max_box_size);
    std::vector<Box> bs;
    for (auto& z : p[2])
        for (auto& y : p[1])
            for (auto& x : p[0]) bs.push_back(Box{{x.first, y.first, z.first}, {x.second, y.second, z.second}});
    return make_ba(dom_lo, dom_hi, bc, std::move(bs), out);
}

bxmg_status bxmg_define_boxarray_list(const int32_t dom_lo[3], const int32_t dom_hi[3], const int32_t bc[3],
                                      int32_t nboxes, const int32_t* lohi, bxmg_boxarray* out) {
    if (!out || !valid_dom(dom_lo, dom_hi)) return fail(BXMG_EINVAL, "define_boxarray_list: empty domain");
    if (nboxes < 1 || !lohi) return fail(BXMG_EINVAL, "define_boxarray_list: no boxes");
    for (int d = 0; d < 3; ++d)
        if (bc && bc[d] != BXMG_PERIODIC && bc[d] != BXMG_DIRICHLET0) return fail(BXMG_EINVAL, "define_boxarray_list: bad bc");
    Box dom{{dom_lo[0], dom_lo[1], dom_lo[2]}, {dom_hi[0], dom_hi[1], dom_hi[2]}};
    std::vector<Box> bs;
    for (int b = 0; b < nboxes; ++b) {
        Box x{{lohi[6 * b], lohi[6 * b + 1], lohi[6 * b + 2]}, {lohi[6 * b + 3], lohi[6 * b + 4], lohi[6 * b + 5]}};
        if (!x.ok()) return fail(BXMG_EINVAL, "define_boxarray_list: empty box " + std::to_string(b));
        if (!dom.contains(x)) return fail(BXMG_EINVAL, "define_boxarray_list: box " + std::to_string(b) + " leaves the domain");
        bs.push_back(x);
    }
    for (size_t a = 0; a < bs.size(); ++a)
        for (size_t b = a + 1; b < bs.size(); ++b)
            if (intersect(bs[a], bs[b]).ok())
                return fail(BXMG_EINVAL, "define_boxarray_list: boxes " + std::to_string(a) + " and " + std::to_string(b) + " overlap");
    return make_ba(dom_lo, dom_hi, bc, std::move(bs), out);
}

bxmg_status bxmg_boxarray_get(bxmg_boxarray ba, int32_t* nboxes, int32_t* lohi_out) {
    if (!ba || !nboxes) return fail(BXMG_EINVAL, "boxarray_get: NULL argument");
    *nboxes = (int32_t)ba->boxes.size();
    if (lohi_out)
        for (size_t b = 0; b < ba->boxes.size(); ++b)
            for (int d = 0; d < 3; ++d) {
                lohi_out[6 * b + d] = ba->boxes[b].lo[d];
                lohi_out[6 * b + 3 + d] = ba->boxes[b].hi[d];
            }
    return BXMG_OK;
}

bxmg_status bxmg_boxarray_hierarchy(bxmg_boxarray ba, int32_t cap_levels, int32_t* nlevels, int32_t* lev_nboxes,
                                    int32_t* lev_dom, int32_t cap_boxes, int32_t* lev_lohi) {
    if (!ba || !nlevels || !lev_nboxes || !lev_dom || !lev_lohi) return fail(BXMG_EINVAL, "boxarray_hierarchy: NULL argument");
    auto L = make_hierarchy(ba->dom, ba->boxes);
    long long tot = 0;
    for (auto& l : L) tot += (long long)l.boxes.size();
    if ((int)L.size() > cap_levels || tot > cap_boxes) return fail(BXMG_EINVAL, "boxarray_hierarchy: capacity too small");
    *nlevels = (int32_t)L.size();
    int o = 0;
    for (size_t l = 0; l < L.size(); ++l) {
        lev_nboxes[l] = (int32_t)L[l].boxes.size();
        for (int d = 0; d < 3; ++d) { lev_dom[6 * l + d] = L[l].dom.lo[d]; lev_dom[6 * l + 3 + d] = L[l].dom.hi[d]; }
        for (auto& b : L[l].boxes) {
            for (int d = 0; d < 3; ++d) { lev_lohi[6 * o + d] = b.lo[d]; lev_lohi[6 * o + 3 + d] = b.hi[d]; }
            ++o;
        }
    }
    return BXMG_OK;
}

void bxmg_boxarray_release(bxmg_boxarray ba) { ba_release(ba); }

size_t bxmg_multifab_bytes(bxmg_boxarray ba, int32_t ncomp, int32_t nghost, bxmg_dtype dtype) {
    if (!ba || ncomp < 1 || nghost < 0 || (dtype != BXMG_F64 && dtype != BXMG_F32)) return 0;
    return mf_layout(ba, ncomp, nghost, dtype, nullptr);
}

bxmg_status bxmg_alloc_multifab(bxmg_ctx ctx, bxmg_boxarray ba, int32_t ncomp, int32_t nghost, bxmg_dtype dtype,
                                void* device_buf, bxmg_multifab* out) {
    if (!ctx || !ba || !out) return fail(BXMG_EINVAL, "alloc_multifab: NULL argument");
    if (ncomp < 1 || nghost < 0) return fail(BXMG_EINVAL, "alloc_multifab: ncomp < 1 or nghost < 0");
    if (dtype != BXMG_F64 && dtype != BXMG_F32) return fail(BXMG_EINVAL, "alloc_multifab: bad dtype");
    if (device_buf && ((uintptr_t)device_buf % 256) != 0) return fail(BXMG_EINVAL, "alloc_multifab: buffer not 256-byte aligned");
    for (int d = 0; d < 3; ++d)
        if (ba->per[d] && nghost > ba->dom.n(d))
            return fail(BXMG_EINVAL, "alloc_multifab: nghost exceeds a periodic domain edge");
    auto mf = std::make_unique<bxmg_mf_s>();
    mf->ctx = ctx;
    mf->ba = ba;
    mf->ncomp = ncomp;
    mf->ng = nghost;
    mf->dtype = dtype;
    mf->bytes = mf_layout(ba, ncomp, nghost, dtype, &mf->fboxes);
    try {
        HIPCHK(hipSetDevice(ctx->device));
        if (device_buf) {
            mf->data = device_buf;
        } else {
            // stream-ordered, so that the release can be too
            if (hipMallocAsync(&mf->data, std::max<size_t>(mf->bytes, 256), ctx->stream) != hipSuccess)
                return fail(BXMG_ENOMEM, "alloc_multifab: hipMallocAsync failed");
            mf->owned = true;
        }
        mf->d_fboxes.upload_async(mf->fboxes, ctx->stream);
    } catch (HipError& e) {
        return fail(BXMG_EDEVICE, std::string("alloc_multifab: ") + hipGetErrorString(e.e));
    }
    ba->refs++;
    *out = mf.release();
    return BXMG_OK;
}

bxmg_status bxmg_multifab_box_view(bxmg_multifab mf, int32_t box, void** dptr, int32_t lo[3], int32_t hi[3],
                                   int64_t strides[4]) {
    if (!mf || !dptr || !lo || !hi || !strides) return fail(BXMG_EINVAL, "box_view: NULL argument");
    if (box < 0 || box >= (int)mf->fboxes.size()) return fail(BXMG_EINVAL, "box_view: box index out of range");
    const FBox& f = mf->fboxes[box];
    const size_t es = (mf->dtype == BXMG_F64) ? 8 : 4;
    *dptr = (char*)mf->data + f.base * es;
    for (int d = 0; d < 3; ++d) { lo[d] = f.glo[d]; hi[d] = f.glo[d] + f.G[d] - 1; }
    strides[0] = 1;
    strides[1] = f.G[0];
    strides[2] = (int64_t)f.G[0] * f.G[1];
    strides[3] = f.cs;
    return BXMG_OK;
}

bxmg_status bxmg_multifab_info(bxmg_multifab mf, void** base, size_t* bytes, int32_t* ncomp, int32_t* nghost,
                               int32_t* dtype) {
    if (!mf) return fail(BXMG_EINVAL, "multifab_info: NULL handle");
    if (base) *base = mf->data;
    if (bytes) *bytes = mf->bytes;
    if (ncomp) *ncomp = mf->ncomp;
    if (nghost) *nghost = mf->ng;
    if (dtype) *dtype = mf->dtype;
    return BXMG_OK;
}

bxmg_status bxmg_multifab_copy_host(bxmg_multifab mf, int32_t to_device, void* host, int32_t comp, void* hip_stream) {
    if (!mf || !host) return fail(BXMG_EINVAL, "multifab_copy_host: NULL argument");
    if (comp < 0 || comp >= mf->ncomp) return fail(BXMG_EINVAL, "multifab_copy_host: component out of range");
    try {
        HIPCHK(hipSetDevice(mf->ctx->device));
        hipStream_t s = hip_stream ? (hipStream_t)hip_stream : mf->ctx->stream;
        std::vector<unsigned char> slab(mf->bytes);
        // the whole slab: ghosts and other components keep their values
        HIPCHK(hipMemcpyAsync(slab.data(), mf->data, mf->bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (mf->dtype == BXMG_F64) copy_valid<double>(mf, slab, (double*)host, comp, to_device != 0);
        else copy_valid<float>(mf, slab, (float*)host, comp, to_device != 0);
        if (to_device) {
            HIPCHK(hipMemcpyAsync(mf->data, slab.data(), mf->bytes, hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
        }
    } catch (HipError& e) {
        return fail(BXMG_EDEVICE, std::string("multifab_copy_host: ") + hipGetErrorString(e.e));
    }
    return BXMG_OK;
}

void bxmg_multifab_release(bxmg_multifab mf) {
    if (!mf) return;
    (void)hipSetDevice(mf->ctx->device);
    const hipStream_t s = mf->ctx->stream;
    if (mf->owned) (void)hipFreeAsync(mf->data, s);
    mf->d_fboxes.release_async(s);
    for (auto& kv : mf->plans) {
        kv.second->tags.release_async(s);
        kv.second->hints.release_async(s);
    }
    for (auto& kv : mf->pcopy_plans) {
        kv.second->tags.release_async(s);
        kv.second->hints.release_async(s);
    }
    ba_release(mf->ba);
    delete mf;
}

static bxmg_status run_fill(bxmg_multifab mf, int32_t scomp, int32_t ncomp, int mode, bool cross, bool odd,
                            void* stream) {
    if (!mf) return fail(BXMG_EINVAL, "fill: NULL MultiFab");
    if (scomp < 0 || ncomp < 1 || scomp + ncomp > mf->ncomp) return fail(BXMG_EINVAL, "fill: component range");
    try {
        HIPCHK(hipSetDevice(mf->ctx->device));
        Plan* p = mf_plan(mf, mode, cross, odd);
        hipStream_t s = stream ? (hipStream_t)stream : mf->ctx->stream;
        HIPCHK(launch_fill_fab(s, mf->data, mf->dtype == BXMG_F32, mf->d_fboxes.p, p->tags.p, p->ntags, p->cells, scomp,
                               ncomp, p->hints.p));
    } catch (HipError& e) {
        return fail(BXMG_EDEVICE, std::string("fill: ") + hipGetErrorString(e.e));
    }
    return BXMG_OK;
}

bxmg_status bxmg_fill_boundary(bxmg_multifab mf, int32_t scomp, int32_t ncomp, int32_t cross, void* hip_stream) {
    return run_fill(mf, scomp, ncomp, 0, cross != 0, false, hip_stream);
}

bxmg_status bxmg_apply_domain_bc(bxmg_multifab mf, int32_t scomp, int32_t ncomp, int32_t odd, void* hip_stream) {
    return run_fill(mf, scomp, ncomp, 1, false, odd != 0, hip_stream);
}

bxmg_status bxmg_parallel_copy(bxmg_multifab dst, int32_t dcomp, bxmg_multifab src, int32_t scomp, int32_t ncomp,
                               int32_t dst_nghost, void* hip_stream) {
    if (!dst || !src) return fail(BXMG_EINVAL, "parallel_copy: NULL MultiFab");
    if (ncomp < 1 || dcomp < 0 || scomp < 0 || dcomp + ncomp > dst->ncomp || scomp + ncomp > src->ncomp)
        return fail(BXMG_EINVAL, "parallel_copy: component range");
    if (dst->dtype != src->dtype) return fail(BXMG_EINVAL, "parallel_copy: dtypes differ");
    if (dst_nghost < 0 || dst_nghost > dst->ng) return fail(BXMG_EINVAL, "parallel_copy: dst_nghost out of [0, nghost]");
    const bxmg_ba_s* db = dst->ba;
    const bxmg_ba_s* sb = src->ba;
    for (int d = 0; d < 3; ++d) {
        if (db->dom.lo[d] != sb->dom.lo[d] || db->dom.hi[d] != sb->dom.hi[d] || db->per[d] != sb->per[d])
            return fail(BXMG_EINVAL, "parallel_copy: the BoxArrays have different domains or boundaries");
        if (db->per[d] && dst_nghost > db->dom.n(d))
            return fail(BXMG_EINVAL, "parallel_copy: dst_nghost exceeds a periodic domain edge");
    }
    if (dst->ctx->device != src->ctx->device) return fail(BXMG_EINVAL, "parallel_copy: different devices");
    try {
        HIPCHK(hipSetDevice(dst->ctx->device));
        const auto key = std::make_pair(sb->id, (int)dst_nghost);
        auto it = dst->pcopy_plans.find(key);
        if (it == dst->pcopy_plans.end()) {
            auto p = std::make_unique<Plan>();
            p->set(pcopy_tags(db->dom, db->per, db->boxes, dst_nghost, sb->boxes), dst->ctx->stream);
            it = dst->pcopy_plans.emplace(key, std::move(p)).first;
        }
        const Plan& P = *it->second;
        hipStream_t s = hip_stream ? (hipStream_t)hip_stream : dst->ctx->stream;
        HIPCHK(launch_copy_fab(s, dst->dtype == BXMG_F32, dst->data, dst->d_fboxes.p, src->data, src->d_fboxes.p,
                               P.tags.p, P.ntags, P.cells, dcomp, scomp, ncomp, P.hints.p));
    } catch (HipError& e) {
        return fail(BXMG_EDEVICE, std::string("parallel_copy: ") + hipGetErrorString(e.e));
    }
    return BXMG_OK;
}

bxmg_status bxmg_fill_boundary_noalloc(bxmg_multifab mf, int32_t scomp, int32_t ncomp, int32_t cross,
                                       void* hip_stream) {
    if (!mf) return fail(BXMG_EINVAL, "fill_noalloc: NULL MultiFab");
    if (scomp < 0 || ncomp < 1 || scomp + ncomp > mf->ncomp) return fail(BXMG_EINVAL, "fill_noalloc: component range");
    // the region list, built once per MultiFab and setting, lives on the host
    const int key = cross ? 2 : 0;
    auto it = mf->host_plans.find(key);
    if (it == mf->host_plans.end()) {
        std::vector<Tag> t = build_tags(mf->ba->dom, mf->ba->per, mf->ba->boxes, mf->ng, cross != 0, 0, false);
        const long long cells = tag_cells(t);
        it = mf->host_plans.emplace(key, std::make_pair(std::move(t), cells)).first;
    }
    const std::vector<Tag>& tags = it->second.first;
    const size_t bytes = tags.size() * sizeof(Tag);
    if (bytes > kScratchBytes)
        return fail(BXMG_EINVAL, "fill_noalloc: " + std::to_string(tags.size()) + " ghost regions need " +
                                     std::to_string(bytes) + " bytes of staging, more than the " +
                                     std::to_string(kScratchBytes) + " available");
    if (tags.empty()) return BXMG_OK;
    try {
        HIPCHK(hipSetDevice(mf->ctx->device));
        hipStream_t s = hip_stream ? (hipStream_t)hip_stream : mf->ctx->stream;
        // staged in stream order: an earlier call's exchange on this stream
        // has read its list before this copy overwrites it
        HIPCHK(hipMemcpyAsync(mf->ctx->scratch, tags.data(), bytes, hipMemcpyHostToDevice, s));
        HIPCHK(launch_fill_fab(s, mf->data, mf->dtype == BXMG_F32, mf->d_fboxes.p, (const Tag*)mf->ctx->scratch,
                               (int)tags.size(), it->second.second, scomp, ncomp, nullptr));
    } catch (HipError& e) {
        return fail(BXMG_EDEVICE, std::string("fill_noalloc: ") + hipGetErrorString(e.e));
    }
    return BXMG_OK;
}

void bxmg_solve_params_default(bxmg_solve_params* p) {
    if (!p) return;
    p->nu1 = 2;
    p->nu2 = 2;
    p->max_cycles = 200;
    p->precision = 0;
    p->prolong = 2;
    p->fixed_cycles = 0;
    p->rel_tol = 1e-10;
    p->abs_tol = 0.0;
    p->dx = 0.0;
    p->bottom_rtol = 1e-12;
    p->krylov = 0;
    p->reserved = 0;
    p->alpha = 0.0;
}

static bxmg_status set_status(bxmg_solve_info* info, bxmg_status st) {
    info->status = st;
    return st;
}

// Hierarchies are cached per geometry (domain, boundary conditions, boxes)
// and settings, so BoxArrays of the same shape share one; the least recently
// used are dropped beyond kCacheEntries entries or kCacheBytes of storage.
constexpr size_t kCacheEntries = 16;
constexpr size_t kCacheBytes = size_t(48) << 30;

static std::string hier_key(const bxmg_ctx_s* ctx, const bxmg_ba_s* ba, int precision, bool var, double h,
                            bool merge, double alpha) {
    std::string k;
    auto put = [&](long long x) { k.append((const char*)&x, sizeof x); };
    long long hb, ab;
    std::memcpy(&hb, &h, sizeof hb);
    std::memcpy(&ab, &alpha, sizeof ab);
    put(ab);
    put(precision);
    put(var);
    put(merge);
    put(hb);
    put(ctx->zc);
    put(ctx->zc_planes);
    put(ctx->res);
    put(ctx->ly_cap);
    for (int d = 0; d < 3; ++d) { put(ba->dom.lo[d]); put(ba->dom.hi[d]); put(ba->per[d]); }
    for (auto& b : ba->boxes)
        for (int d = 0; d < 3; ++d) { put(b.lo[d]); put(b.hi[d]); }
    return k;
}

static void cache_touch(bxmg_ctx ctx, const std::string& key) {
    for (auto it = ctx->lru.begin(); it != ctx->lru.end(); ++it)
        if (*it == key) { ctx->lru.erase(it); break; }
    ctx->lru.push_back(key);
}

static void cache_trim(bxmg_ctx ctx, const std::string& keep) {
    auto total = [&]() {
        size_t t = 0;
        for (auto& e : ctx->cache) t += e.second->bytes;
        return t;
    };
    while (ctx->lru.size() > 1 && (ctx->lru.size() > kCacheEntries || total() > kCacheBytes)) {
        const std::string victim = ctx->lru.front();
        if (victim == keep) break;
        ctx->lru.pop_front();
        ctx->cache.erase(victim);
    }
}

static Hier* get_hier(bxmg_ctx ctx, const bxmg_ba_s* ba, int precision, bool var, double h, bxmg_status* st,
                      bool merge = true, double alpha = 0.0) {
    const std::string key = hier_key(ctx, ba, precision, var, h, merge, alpha);
    auto it = ctx->cache.find(key);
    if (it != ctx->cache.end()) {
        cache_touch(ctx, key);
        return it->second.get();
    }
    auto lb = make_hierarchy(ba->dom, ba->boxes);
    const LevelBoxes& bot = lb.back();
    if (!bottom_fits(bot.dom)) {
        *st = fail(BXMG_EINVAL, "solve: bottom level has " + std::to_string(bot.dom.cells()) +
                                    " cells (at most 4096, and 6144 with its ghost layer)");
        return nullptr;
    }
    std::unique_ptr<Hier> H;
    try {
        Tuning tune;
        tune.zc = ctx->zc;
        tune.zc_planes = ctx->zc_planes;
        tune.res = ctx->res;
        tune.ly_cap = ctx->ly_cap;
        H = build_hier(ba, precision, var, h, tune, merge, alpha);
    } catch (HipError& e) {
        *st = fail(e.e == hipErrorOutOfMemory ? BXMG_ENOMEM : BXMG_EDEVICE,
                   std::string("solve: hierarchy setup: ") + e.where + ": " + hipGetErrorString(e.e));
        return nullptr;
    } catch (std::exception& e) {
        *st = fail(BXMG_EINVAL, std::string("solve: hierarchy setup: ") + e.what());
        return nullptr;
    }
    Hier* raw = H.get();
    ctx->cache[key] = std::move(H);
    cache_touch(ctx, key);
    cache_trim(ctx, key);
    return raw;
}

// Multigrid-preconditioned conjugate gradients on level 0 (reading R23):
// flexible CG, one V-cycle from zero per iteration as the preconditioner
// (FP32 with its FP64 bottom, or FP64), every scalar on the device.  On
// entry level 0 holds u (with current face ghosts) and f, and the slot is
// admitted; on return u is in level 0's FP64 array and the stop test's
// history in the slot.  Per iteration:
//   p' = z + beta p (every element), q = L p', alpha = rz / (p'.q)
//   u += alpha p', r -= alpha q, stop test on |r|_inf     (update pass)
//   z = M r                                               (the V-cycle)
//   beta = -alpha (z.q) / rz, rz = z.r                    (dot pass)
// When the updated residual meets the tolerance, f - L u is computed afresh;
// if that misses it, the iteration restarts from it (p = z = M r).
static void krylov_iterate(Run& R, Hier* H, const bxmg_solve_params& P, bxmg_ctx ctx, SolveState* hs, bool var,
                           int limit, const std::function<void()>& look, const std::function<int(int, int)>& predict,
                           double* true_inf, double* true_l2) {
    const Level& L0 = *H->L[0];
    const long long n = L0.nelem;
    Hier::Krylov& K = H->kr;
    if (!K.r.p) {
        K.r.alloc(n);
        K.q.alloc(n);
        K.p[0].alloc(n);
        K.p[1].alloc(n);
        K.part.alloc(3 * (size_t)std::max(L0.ntcol, 1));
        K.sums.alloc(3);
        K.sc.alloc(1);
        HIPCHK(hipMemsetAsync(K.sc.p, 0, sizeof(KrylovScalars), R.s));
        // ghosts of r are never written, q is read before its first write
        // (a restart's dot pass discards z.q): both start at zero
        HIPCHK(launch_zero<double>(R.s, K.r.p, n));
        HIPCHK(launch_zero<double>(R.s, K.q.p, n));
        H->bytes += 32 * (size_t)n;
    }
    const bool fp32 = P.precision == 1;
    double* u = H->u64[0]->p;
    double* x = u;
    const double* f = H->f64[0]->p;
    if (!fp32) {
        // the FP64 V-cycle works in level 0's own arrays: the iterate and the
        // right-hand side move out for the solve
        if (!K.x.p) {
            K.x.alloc(n);
            K.f.alloc(n);
            H->bytes += 16 * (size_t)n;
        }
        HIPCHK(hipMemcpyAsync(K.x.p, u, n * sizeof(double), hipMemcpyDeviceToDevice, R.s));
        HIPCHK(hipMemcpyAsync(K.f.p, H->f64[0]->p, n * sizeof(double), hipMemcpyDeviceToDevice, R.s));
        x = K.x.p;
        f = K.f.p;
    }
    const double* b64 = var ? H->beta64.p : nullptr;
    const FaceArrays<double>* nf = nullptr;
    double* pc = K.p[0].p;
    double* pn = K.p[1].p;
    HIPCHK(launch_zero<double>(R.s, pc, n));  // beta = 0 reads it: keep it finite
    HIPCHK(launch_zero<double>(R.s, pn, n));
    Run R0 = R;  // the same, with launches that run whatever the stop flag says
    R0.active = nullptr;
    auto stop_test = [&]() {
        HIPCHK(launch_norm_final(R.s, H->partials.p, L0.ntcol, H->fnorm.p));
        HIPCHK(launch_batch_check(R.s, H->flags.p + 1, 1, H->fnorm.p, H->st.p, H->flags.p, H->hist.p,
                                  H->hist.p + kHist, H->flags.p + 2));
    };
    // z = M r, from the right-hand side already in place; zero: clear the
    // correction first (the direction pass clears it on the way otherwise)
    auto precondition = [&](bool zero) {
        if (fp32) {
            if (zero) HIPCHK(launch_zero<float>(R.s, H->u32[0]->p, n, R.active));
            vcycle<float>(R, 0);
            fill_faces<float>(R, 0, H->u32[0]->p);
        } else {
            if (zero) HIPCHK(launch_zero<double>(R.s, H->u64[0]->p, n, R.active));
            vcycle<double>(R, 0);
            fill_faces<double>(R, 0, H->u64[0]->p);
        }
    };
    auto dots = [&](int step) {
        if (fp32) HIPCHK(launch_kr_dots<float>(R.s, R.grid(L0.walk()), H->u32[0]->p, K.r.p, K.q.p, K.part.p));
        else HIPCHK(launch_kr_dots<double>(R.s, R.grid(L0.walk()), H->u64[0]->p, K.r.p, K.q.p, K.part.p));
        HIPCHK(launch_norm_final(R.s, K.part.p, L0.ntcol, K.sums.p));
        HIPCHK(launch_kr_step(R.s, K.sums.p, K.sc.p, step, R.active));
    };
    // f - L u into r (and its norms into the partials); u's ghosts refreshed first
    auto residual = [&](Run& Rx, const Grid& g) {
        fill_faces<double>(Rx, 0, x);
        HIPCHK(launch_resid<double, double>(R.s, g, x, f, b64, nf, K.r.p, H->partials.p));
    };
    auto restart = [&]() {  // p = z = M r
        if (fp32) HIPCHK(launch_cast_f32(R.s, K.r.p, H->f32[0]->p, n));
        else HIPCHK(hipMemcpyAsync(H->f64[0]->p, K.r.p, n * sizeof(double), hipMemcpyDeviceToDevice, R.s));
        precondition(true);
        dots(2);
    };
    auto iterate = [&]() {
        if (fp32) HIPCHK(launch_kr_axpy<float>(R.s, H->u32[0]->p, pc, pn, n, K.sc.p, R.active));
        else HIPCHK(launch_kr_axpy<double>(R.s, H->u64[0]->p, pc, pn, n, K.sc.p, R.active));
        std::swap(pc, pn);
        HIPCHK(launch_kr_apply(R.s, R.grid(L0.walk()), pc, b64, K.q.p, K.part.p));
        HIPCHK(launch_norm_final(R.s, K.part.p, L0.ntcol, K.sums.p));
        HIPCHK(launch_kr_step(R.s, K.sums.p, K.sc.p, 0, R.active));
        if (fp32)
            HIPCHK(launch_kr_update<float>(R.s, R.grid(L0.walk()), x, pc, K.r.p, K.q.p, H->f32[0]->p, K.sc.p,
                                           H->partials.p));
        else
            HIPCHK(launch_kr_update<double>(R.s, R.grid(L0.walk()), x, pc, K.r.p, K.q.p, H->f64[0]->p, K.sc.p,
                                            H->partials.p));
        stop_test();
        precondition(false);
        dots(1);
    };
    residual(R, R.grid(L0.walk()));
    stop_test();
    int queued = 0;
    if (limit > 0) {
        restart();
        iterate();
        queued = 1;
    }
    for (;;) {
        look();
        if (hs->active) {
            const int ahead = predict(queued, limit);
            for (int a = 0; a < ahead; ++a) {
                iterate();
                ++queued;
            }
            continue;
        }
        if (hs->st.status != 0 || hs->st.nhist == 0) break;  // no convergence, non-finite, or not admitted
        // the updated residual met the test: take f - L u itself
        residual(R0, L0.grid());
        HIPCHK(launch_norm_final(R.s, H->partials.p, L0.ntcol, H->fnorm.p));
        HIPCHK(hipMemcpyAsync(ctx->h_norm, H->fnorm.p, 3 * sizeof(double), hipMemcpyDeviceToHost, R.s));
        HIPCHK(hipStreamSynchronize(R.s));
        const double tinf = ctx->h_norm[2] > 0.0 ? (double)NAN : ctx->h_norm[0];
        *true_inf = tinf;
        *true_l2 = std::sqrt(ctx->h_norm[1]);
        const double fn = hs->st.fnorm;
        if (P.fixed_cycles > 0 || !(tinf == tinf) || tinf <= P.rel_tol * fn || tinf <= P.abs_tol) break;
        if (hs->st.cycles >= limit) {  // no room left to restart
            hs->st.status = BXMG_ENOCONV;
            break;
        }
        // restart from the fresh residual (already in r): the slot runs on
        hs->st.cycles += 1;
        hs->active = 1;
        HIPCHK(hipMemcpyAsync(H->st.p, &hs->st, sizeof(BatchSlot), hipMemcpyHostToDevice, R.s));
        HIPCHK(hipMemcpyAsync(H->flags.p, &hs->active, sizeof(int), hipMemcpyHostToDevice, R.s));
        restart();
        iterate();
        queued = hs->st.cycles;
    }
    if (!fp32) HIPCHK(hipMemcpyAsync(u, x, n * sizeof(double), hipMemcpyDeviceToDevice, R.s));
}

// A solve; heat_dt > 0 makes it a backward-Euler heat step: the right-hand
// side is formed on the device from phi (the state) and src (NULL: no
// source) as f = -(phi * (1/dt) + src), and alpha = 1/dt (reading R24).
static bxmg_status solve_impl(bxmg_ctx ctx, const bxmg_solve_params* params, bxmg_multifab phi, bxmg_multifab rhs,
                              bxmg_multifab beta, bxmg_solve_info* info, double heat_dt, bxmg_multifab src) {
    const bool heat = heat_dt > 0.0;
    if (!ctx || !phi || (!rhs && !heat) || !info) return fail(BXMG_EINVAL, "solve: NULL argument");
    std::memset(info, 0, sizeof(*info));
    bxmg_solve_params P;
    if (params) P = *params;
    else bxmg_solve_params_default(&P);
    const double inv_dt = heat ? 1.0 / heat_dt : 0.0;
    if (heat) P.alpha = inv_dt;
    const bxmg_ba_s* ba = phi->ba;
    bxmg_status st;
    if ((st = check_solve_mf(phi, ba, "phi")) != BXMG_OK) return set_status(info, st);
    if (!heat && (st = check_solve_mf(rhs, ba, "rhs")) != BXMG_OK) return set_status(info, st);
    if (src && (st = check_field_mf(src, ba, "source")) != BXMG_OK) return set_status(info, st);
    if (beta && (st = check_solve_mf(beta, ba, "beta")) != BXMG_OK) return set_status(info, st);
    if (!covers_domain(ba)) return set_status(info, fail(BXMG_EINVAL, "solve: the BoxArray must cover its domain"));
    if (P.nu1 < 0 || P.nu2 < 0 || P.max_cycles < 0 || (P.precision != 0 && P.precision != 1) ||
        (P.prolong != 1 && P.prolong != 2) || (P.krylov != 0 && P.krylov != 1) ||
        !(P.alpha >= 0.0 && P.alpha <= 1.7976931348623157e308))
        return set_status(info, fail(BXMG_EINVAL, "solve: bad parameters"));
    const double h = (P.dx > 0) ? P.dx : 1.0 / ba->dom.n(0);
    std::lock_guard<std::mutex> lock(ctx->mu);
    const auto t0 = std::chrono::steady_clock::now();
    try {
        HIPCHK(hipSetDevice(ctx->device));
        st = BXMG_OK;
        Hier* H = get_hier(ctx, ba, P.precision, beta != nullptr, h, &st, ctx->merge != 0, P.alpha);
        if (!H) return set_status(info, st);
        info->levels = (int)H->L.size();
        Run R{H, ctx->stream, P.nu1, P.nu2, P.prolong, P.bottom_rtol};
        R.prof = &ctx->prof;
        R.lds_coarse = ctx->lds_coarse != 0;
        const Level& L0 = *H->L[0];
        double* u = H->u64[0]->p;
        double* f = H->f64[0]->p;
        // caller layout -> colour-split level 0; flags[3] = whether the guess
        // has a value other than +0.0 (the first residual skips the reads of
        // an all-zero guess)
        int* const guess_nz = H->flags.p + 3;
        HIPCHK(hipMemsetAsync(guess_nz, 0, sizeof(int), R.s));
        HIPCHK(launch_fab_to_rb_nz(R.s, L0.view_grid(), (const double*)phi->data, phi->d_fboxes.p, u, guess_nz));
        // f, with the norms of f per tile on the way (reduced below)
        if (heat)
            HIPCHK(launch_heat_rhs(R.s, L0.view_grid(), (const double*)phi->data, phi->d_fboxes.p,
                                   src ? (const double*)src->data : nullptr, src ? src->d_fboxes.p : nullptr, inv_dt,
                                   f, H->partials.p));
        else
            HIPCHK(launch_fab_to_rb_norm(R.s, L0.view_grid(), (const double*)rhs->data, rhs->d_fboxes.p, f,
                                         H->partials.p));
        if (beta) {
            HIPCHK(launch_fab_to_rb(R.s, L0.view_grid(), (const double*)beta->data, beta->d_fboxes.p, H->beta64.p, false));
            if (P.precision == 0) {
                setup_faces<double>(R, H->beta64.p);
            } else {
                fill<double>(R, 0, H->beta64.p, L0.full_even);
                HIPCHK(launch_cast_f32(R.s, H->beta64.p, H->beta32.p, L0.nelem));
                setup_faces<float>(R, H->beta32.p);
            }
        }
        // ghost cells of the converted guess; from here on every producer of
        // level-0 values refreshes the face ghosts it mirrors (push levels)
        fill_faces<double>(R, 0, u);
        const FaceArrays<double>* nf = nullptr;
        // The stop test runs on the device (the batch engine's, for one
        // slot): k_batch_admit takes the norm of f, and k_batch_check after
        // every residual records the history and clears the active flag once
        // the solve stops (converged, max_cycles, fixed_cycles, non-finite).
        // Every kernel of a V-cycle honours the flag, so the host enqueues
        // cycles ahead of the device and reads the state back only now and
        // then, instead of once per cycle.
        SolveState* hs = (SolveState*)ctx->h_solve;
        BatchSlot S0{};
        S0.rel_tol = P.rel_tol;
        S0.abs_tol = P.abs_tol;
        S0.max_cycles = P.max_cycles;
        S0.fixed_cycles = P.fixed_cycles;
        hs->st = S0;  // pinned: the source of the copy
        HIPCHK(hipMemcpyAsync(H->st.p, &hs->st, sizeof S0, hipMemcpyHostToDevice, R.s));
        HIPCHK(launch_norm_final(R.s, H->partials.p, L0.view_grid().ntiles, H->fn3.p));
        HIPCHK(launch_batch_admit(R.s, H->fn3.p, H->st.p, H->flags.p, 0));
        R.active = H->flags.p;
        // FP64 solves on a pushing, buffer-addressed level 0 with post-smoothing
        // take the colour-1 residual norms in the V-cycle's last level-0 sweep
        const bool fusable = P.precision == 0 && L0.push && L0.res && P.nu2 > 0;
        double* const norms1 = H->partials.p + 3 * (size_t)L0.ntcol;
        const int* first_nz = guess_nz;  // for the first residual only
        auto check = [&](bool fused) {  // residual of the current iterate, then the stop test
            if (!L0.push) fill_faces<double>(R, 0, u);
            R.pre(0, kStageResid);
            if (fused) {
                // colour 0 now; colour 1's norms are in the second set
                HIPCHK(launch_resid<double, double>(R.s, R.grid(L0.walk()), u, f, beta ? H->beta64.p : nullptr, nf,
                                                    (double*)nullptr, H->partials.p, true));
            } else if (P.precision == 0) {
                HIPCHK(launch_resid<double, double>(R.s, R.grid(L0.walk()), u, f, beta ? H->beta64.p : nullptr, nf,
                                                    (double*)nullptr, H->partials.p, false, first_nz));
            } else {
                HIPCHK(launch_resid<double, float>(R.s, R.grid(L0.walk()), u, f, beta ? H->beta64.p : nullptr, nf,
                                                   H->f32[0]->p, H->partials.p, false, first_nz));
            }
            first_nz = nullptr;
            R.post(0, kStageResid);
            HIPCHK(launch_norm_final(R.s, H->partials.p, (fused ? 2 : 1) * L0.ntcol, H->fnorm.p));
            HIPCHK(launch_batch_check(R.s, H->flags.p + 1, 1, H->fnorm.p, H->st.p, H->flags.p, H->hist.p,
                                      H->hist.p + kHist, H->flags.p + 2));
        };
        auto cycle = [&]() {  // returns whether its last level-0 sweep took the colour-1 norms
            if (P.precision == 0) {
                R.fuse_norms = fusable ? norms1 : nullptr;
                R.fused_sweep = false;
                vcycle<double>(R, 0);
                R.fuse_norms = nullptr;
                return R.fused_sweep;
            } else {
                HIPCHK(launch_zero<float>(R.s, H->u32[0]->p, L0.nelem, R.active));
                vcycle<float>(R, 0);
                HIPCHK(launch_add_f32(R.s, R.grid(L0.walk()), u, H->u32[0]->p));
                return false;
            }
        };
        auto look = [&]() {
            HIPCHK(hipMemcpyAsync(hs->hist, H->hist.p, 2 * kHist * sizeof(double), hipMemcpyDeviceToHost, R.s));
            HIPCHK(hipMemcpyAsync(&hs->st, H->st.p, sizeof(BatchSlot), hipMemcpyDeviceToHost, R.s));
            HIPCHK(hipMemcpyAsync(&hs->active, H->flags.p, sizeof(int), hipMemcpyDeviceToHost, R.s));
            HIPCHK(hipStreamSynchronize(R.s));
        };
        // cycles to enqueue ahead of the device, predicted from the history:
        // as many as still seem needed, less one, so that a solve rarely runs
        // on into cycles that do nothing
        auto predict = [&](int queued, int limit) {
            int ahead = limit - queued;
            if (P.fixed_cycles <= 0) {
                int pred = 1;
                const int c = queued;
                if (c >= 1 && c < kHist && hs->st.fnorm > 0.0) {
                    const double r1 = hs->hist[c], rho = r1 / hs->hist[c - 1];
                    const double t = std::max(P.rel_tol, P.abs_tol / hs->st.fnorm);
                    if (rho > 0.0 && rho < 1.0 && r1 > t && t > 0.0)
                        pred = (int)std::min(32.0, std::max(1.0, std::ceil(std::log(t / r1) / std::log(rho)) - 1.0));
                }
                ahead = std::min(ahead, pred);
            }
            return std::max(ahead, 1);
        };
        const int limit = P.fixed_cycles > 0 ? P.fixed_cycles : P.max_cycles;
        double true_inf = -1.0, true_l2 = 0.0;  // f - L u at the end (Krylov solves), when taken
        if (P.krylov) {
            krylov_iterate(R, H, P, ctx, hs, beta != nullptr, limit, look, predict, &true_inf, &true_l2);
        } else {
        // queued = V-cycles enqueued; residual number c follows cycle c
        check(false);
        int queued = 0;
        if (limit > 0) {
            check(cycle());
            queued = 1;
        }
        for (;;) {
            look();
            if (!hs->active) break;
            // the device wants cycle queued + 1
            const int ahead = predict(queued, limit);
            for (int a = 0; a < ahead; ++a) {
                check(cycle());
                ++queued;
            }
        }
        }
        const BatchSlot& Sf = hs->st;
        info->f_inf = Sf.fnorm;
        const int nh = std::min(Sf.nhist, kHist);
        for (int c = 0; c < nh; ++c) {
            info->hist[c] = hs->hist[c];
            info->hist_l2[c] = hs->hist_l2[c];
        }
        info->nhist = nh;
        if (nh > 0) {
            info->rel_resid_inf = hs->hist[nh - 1];
            info->resid_l2 = hs->hist_l2[nh - 1];
        }
        if (true_inf >= 0.0 && Sf.fnorm > 0.0) {  // a Krylov solve's closing f - L u
            info->rel_resid_inf = true_inf / Sf.fnorm;
            info->resid_l2 = true_l2;
        }
        info->cycles = Sf.cycles;
        const int status = Sf.status;
        if (status == BXMG_ENONFINITE && nh == 0) {  // rejected at admission: phi is left as it was
            info->f_inf = NAN;
            ctx->prof.harvest();
            return set_status(info, fail(BXMG_ENONFINITE, "solve: non-finite right-hand side"));
        }
        if (Sf.fnorm == 0.0 && status == 0)  // f == 0: the solution is u = 0 (reading R13)
            HIPCHK(launch_zero<double>(R.s, u, L0.nelem));
        if (ba->per[0] && ba->per[1] && ba->per[2] && P.alpha == 0.0)
            HIPCHK(launch_mean_sub(R.s, L0.mean_grid(), u, H->partials.p));
        HIPCHK(launch_rb_to_fab(R.s, L0.view_grid(), u, (double*)phi->data, phi->d_fboxes.p));
        HIPCHK(hipStreamSynchronize(R.s));
        ctx->prof.harvest();
        info->status = status;
        if (status == BXMG_ENOCONV) fail(BXMG_ENOCONV, "solve: max_cycles reached");
        if (status == BXMG_ENONFINITE) fail(BXMG_ENONFINITE, "solve: non-finite residual");
    } catch (HipError& e) {
        return set_status(info, fail(BXMG_EDEVICE, std::string("solve: ") + e.where + ": " + hipGetErrorString(e.e)));
    }
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return (bxmg_status)info->status;
}

}  // extern "C"

std::shared_ptr<Hier> hier_create(bxmg_ctx ctx, const bxmg_ba_s* ba, double h) {
    auto lb = make_hierarchy(ba->dom, ba->boxes);
    if (!bottom_fits(lb.back().dom)) throw std::runtime_error("bottom level too large");
    Tuning tune;
    tune.zc = ctx->zc;
    tune.zc_planes = ctx->zc_planes;
    tune.res = ctx->res;
    tune.ly_cap = ctx->ly_cap;
    return std::shared_ptr<Hier>(build_hier(ba, 0, false, h, tune, ctx->merge != 0, 0.0).release());
}

void hier_level0(Hier* H, double** u, double** f, RBox* box, int* levels) {
    const Level& L0 = *H->L[0];
    *u = H->u64[0]->p;
    *f = H->f64[0]->p;
    *box = L0.rb.at(0);
    *levels = (int)H->L.size();
}

void hier_vcycle_from_zero(bxmg_ctx ctx, Hier* H, const bxmg_solve_params& P) {
    std::lock_guard<std::mutex> lock(ctx->mu);
    Run R{H, ctx->stream, P.nu1, P.nu2, P.prolong, P.bottom_rtol};
    R.prof = &ctx->prof;
    R.lds_coarse = ctx->lds_coarse != 0;
    const Level& L0 = *H->L[0];
    HIPCHK(launch_zero<double>(R.s, H->u64[0]->p, L0.nelem));
    vcycle<double>(R, 0);
    ctx->prof.harvest();
}

extern "C" {

bxmg_status bxmg_mlmg_solve(bxmg_ctx ctx, const bxmg_solve_params* params, bxmg_multifab phi, bxmg_multifab rhs,
                            bxmg_multifab beta, bxmg_solve_info* info) {
    return solve_impl(ctx, params, phi, rhs, beta, info, 0.0, nullptr);
}

bxmg_status bxmg_heat_step(bxmg_ctx ctx, const bxmg_solve_params* params, bxmg_multifab u, bxmg_multifab source,
                           bxmg_multifab beta, double dt, bxmg_solve_info* info) {
    if (!(dt > 0.0 && dt <= 1.7976931348623157e308)) {
        if (info) std::memset(info, 0, sizeof(*info));
        return info ? set_status(info, fail(BXMG_EINVAL, "heat_step: dt must be positive and finite"))
                    : fail(BXMG_EINVAL, "heat_step: dt must be positive and finite");
    }
    return solve_impl(ctx, params, u, nullptr, beta, info, dt, source);
}


bxmg_status bxmg_ctx_tune(bxmg_ctx ctx, int32_t param, int32_t value) {
    if (!ctx) return fail(BXMG_EINVAL, "ctx_tune: NULL context");
    if (param < 0 || param > 5) return fail(BXMG_EINVAL, "ctx_tune: unknown parameter");
    if (param <= 1 && (value < 1 || value > 64)) return fail(BXMG_EINVAL, "ctx_tune: value out of range [1, 64]");
    if ((param == 2 || param >= 4) && value != 0 && value != 1) return fail(BXMG_EINVAL, "ctx_tune: value must be 0 or 1");
    if (param == 3 && (value < 0 || value > 8)) return fail(BXMG_EINVAL, "ctx_tune: value out of range [0, 8]");
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (param == 0) ctx->zc = value;
    else if (param == 1) ctx->zc_planes = value;
    else if (param == 2) ctx->res = value;
    else if (param == 3) ctx->ly_cap = value;
    else if (param == 4) ctx->lds_coarse = value;
    else ctx->merge = value;
    return BXMG_OK;
}

bxmg_status bxmg_autotune(bxmg_ctx ctx, const bxmg_solve_params* params, bxmg_multifab phi, bxmg_multifab rhs,
                          bxmg_multifab beta, int32_t cycles, int32_t best[4], double* best_ms, int32_t* ntried) {
    if (!ctx || !phi || !rhs) return fail(BXMG_EINVAL, "autotune: NULL argument");
    if (cycles < 1 || cycles > 64) return fail(BXMG_EINVAL, "autotune: cycles out of [1, 64]");
    bxmg_solve_params P;
    if (params) P = *params;
    else bxmg_solve_params_default(&P);
    P.fixed_cycles = cycles;
    // candidates: planes per thread x tile rows x addressing
    const int zcs[] = {1, 2, 4, 8};
    const int lys[] = {2, 3, 8};
    const int ress[] = {1, 0};
    int prev[4];
    {
        std::lock_guard<std::mutex> lock(ctx->mu);
        prev[0] = ctx->zc;
        prev[1] = ctx->res;
        prev[2] = ctx->ly_cap;
        prev[3] = ctx->zc_planes;
    }
    double best_t = 1e300;
    int bz = prev[0], bl = prev[2], br = prev[1], n = 0;
    bxmg_solve_info info;
    for (int zc : zcs)
        for (int ly : lys)
            for (int res : ress) {
                {
                    std::lock_guard<std::mutex> lock(ctx->mu);
                    ctx->zc = ctx->zc_planes = zc;
                    ctx->ly_cap = ly;
                    ctx->res = res;
                }
                bxmg_status st = bxmg_mlmg_solve(ctx, &P, phi, rhs, beta, &info);  // builds the hierarchy
                if (st != BXMG_OK && st != BXMG_ENOCONV) return st;
                double t = 1e300;
                for (int rep = 0; rep < 2; ++rep) {
                    st = bxmg_mlmg_solve(ctx, &P, phi, rhs, beta, &info);
                    if (st != BXMG_OK && st != BXMG_ENOCONV) return st;
                    t = std::min(t, info.seconds);
                }
                ++n;
                if (t < best_t) { best_t = t; bz = zc; bl = ly; br = res; }
            }
    {
        std::lock_guard<std::mutex> lock(ctx->mu);
        ctx->zc = ctx->zc_planes = bz;
        ctx->ly_cap = bl;
        ctx->res = br;
    }
    if (best) { best[0] = bz; best[1] = bz; best[2] = br; best[3] = bl; }
    if (best_ms) *best_ms = best_t * 1000.0 / cycles;
    if (ntried) *ntried = n;
    return BXMG_OK;
}

bxmg_status bxmg_profile_stage(bxmg_ctx ctx, int32_t stage) {
    if (!ctx) return fail(BXMG_EINVAL, "profile_stage: NULL context");
    if (stage < -1 || stage > kStageCoarse) return fail(BXMG_EINVAL, "profile_stage: unknown stage");
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->prof.stage = stage;
    ctx->prof.n = 0;
    return BXMG_OK;
}

bxmg_status bxmg_profile_read(bxmg_ctx ctx, int64_t* launches, double* total_ms, int32_t reset) {
    if (!ctx) return fail(BXMG_EINVAL, "profile_read: NULL context");
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (launches) *launches = ctx->prof.launches;
    if (total_ms) *total_ms = ctx->prof.ms;
    if (reset) { ctx->prof.launches = 0; ctx->prof.ms = 0.0; }
    return BXMG_OK;
}

// ----------------------------------------------------- single-level stages
// Each stage runs the solver's own kernels on the hierarchy cached for the
// caller's BoxArray: caller MultiFabs are converted into the colour-split
// level storage, the stage kernel runs, and the result is converted back.
static bxmg_status stage_prepare(bxmg_ctx ctx, bxmg_multifab phi, bxmg_multifab rhs, bxmg_multifab beta, double h,
                                 Hier** Hout) {
    if (!ctx || !phi) return fail(BXMG_EINVAL, "stage: NULL argument");
    bxmg_status st;
    if ((st = check_solve_mf(phi, phi->ba, "phi")) != BXMG_OK) return st;
    if (rhs && (st = check_solve_mf(rhs, phi->ba, "rhs")) != BXMG_OK) return st;
    if (beta && (st = check_solve_mf(beta, phi->ba, "beta")) != BXMG_OK) return st;
    if (!(h > 0)) return fail(BXMG_EINVAL, "stage: h must be positive");
    st = BXMG_OK;
    Hier* H = get_hier(ctx, phi->ba, 0, beta != nullptr, h, &st, false);
    if (!H) return st;
    *Hout = H;
    return BXMG_OK;
}

static void stage_load(Run& R, Hier* H, bxmg_multifab phi, bxmg_multifab rhs, bxmg_multifab beta) {
    const Level& L0 = *H->L[0];
    HIPCHK(launch_fab_to_rb(R.s, L0.grid(), (const double*)phi->data, phi->d_fboxes.p, H->u64[0]->p, false));
    if (rhs) HIPCHK(launch_fab_to_rb(R.s, L0.grid(), (const double*)rhs->data, rhs->d_fboxes.p, H->f64[0]->p, false));
    if (beta) {
        HIPCHK(launch_fab_to_rb(R.s, L0.grid(), (const double*)beta->data, beta->d_fboxes.p, H->beta64.p, false));
        setup_faces<double>(R, H->beta64.p);
    }
}

bxmg_status bxmg_gs_colour(bxmg_ctx ctx, bxmg_multifab phi, bxmg_multifab rhs, bxmg_multifab beta, double h,
                           int32_t colour) {
    if (colour != 0 && colour != 1) return fail(BXMG_EINVAL, "gs_colour: colour must be 0 or 1");
    if (!rhs) return fail(BXMG_EINVAL, "gs_colour: rhs is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    try {
        HIPCHK(hipSetDevice(ctx->device));
        Hier* H;
        bxmg_status st = stage_prepare(ctx, phi, rhs, beta, h, &H);
        if (st != BXMG_OK) return st;
        Run R{H, ctx->stream, 0, 0, 2, 1e-12};
        stage_load(R, H, phi, rhs, beta);
        const Level& L0 = *H->L[0];
        fill<double>(R, 0, H->u64[0]->p, L0.face[colour ^ 1]);
        HIPCHK(launch_gs<double>(R.s, L0.grid(), H->u64[0]->p, H->f64[0]->p, beta ? H->beta64.p : nullptr,
                                 nullptr, colour));
        HIPCHK(launch_rb_to_fab(R.s, L0.grid(), H->u64[0]->p, (double*)phi->data, phi->d_fboxes.p));
        HIPCHK(hipStreamSynchronize(R.s));
    } catch (HipError& e) {
        return fail(BXMG_EDEVICE, std::string("gs_colour: ") + e.where + ": " + hipGetErrorString(e.e));
    }
    return BXMG_OK;
}

bxmg_status bxmg_residual(bxmg_ctx ctx, bxmg_multifab phi, bxmg_multifab rhs, bxmg_multifab beta, double h,
                          bxmg_multifab r, double norms[2]) {
    if (!rhs || !r) return fail(BXMG_EINVAL, "residual: rhs or r is NULL");
    if (r->ba != phi->ba && check_solve_mf(r, phi->ba, "r") != BXMG_OK) return BXMG_EINVAL;
    if (r->dtype != BXMG_F64) return fail(BXMG_EINVAL, "residual: r must be FP64");
    std::lock_guard<std::mutex> lock(ctx->mu);
    try {
        HIPCHK(hipSetDevice(ctx->device));
        Hier* H;
        bxmg_status st = stage_prepare(ctx, phi, rhs, beta, h, &H);
        if (st != BXMG_OK) return st;
        Run R{H, ctx->stream, 0, 0, 2, 1e-12};
        stage_load(R, H, phi, rhs, beta);
        const Level& L0 = *H->L[0];
        fill_faces<double>(R, 0, H->u64[0]->p);
        // r overwrites f in place (each cell reads its own f, then stores r)
        HIPCHK(launch_resid<double, double>(R.s, L0.grid(), H->u64[0]->p, H->f64[0]->p, beta ? H->beta64.p : nullptr,
                                            nullptr, H->f64[0]->p, H->partials.p));
        HIPCHK(launch_norm_final(R.s, H->partials.p, L0.ntcol, H->fnorm.p));
        HIPCHK(launch_rb_to_fab(R.s, L0.grid(), H->f64[0]->p, (double*)r->data, r->d_fboxes.p));
        norm_readback(R, ctx->h_norm, H->fnorm.p);
        if (norms) {
            norms[0] = ctx->h_norm[2] > 0 ? NAN : ctx->h_norm[0];
            norms[1] = ctx->h_norm[1];
        }
    } catch (HipError& e) {
        return fail(BXMG_EDEVICE, std::string("residual: ") + e.where + ": " + hipGetErrorString(e.e));
    }
    return BXMG_OK;
}

static bool same_boxes(const std::vector<Box>& a, const std::vector<Box>& b) {
    return a.size() == b.size() && std::memcmp(a.data(), b.data(), a.size() * sizeof(Box)) == 0;
}

bxmg_status bxmg_restrict(bxmg_ctx ctx, bxmg_multifab fine, bxmg_multifab coarse) {
    if (!ctx || !fine || !coarse) return fail(BXMG_EINVAL, "restrict: NULL argument");
    std::lock_guard<std::mutex> lock(ctx->mu);
    try {
        HIPCHK(hipSetDevice(ctx->device));
        Hier* H;
        bxmg_status st = stage_prepare(ctx, fine, nullptr, nullptr, 1.0, &H);
        if (st != BXMG_OK) return st;
        if (H->L.size() < 2 || !same_boxes(H->L[1]->boxes, coarse->ba->boxes))
            return fail(BXMG_EINVAL, "restrict: coarse BoxArray is not the next level of the fine one");
        if ((st = check_solve_mf(coarse, coarse->ba, "coarse")) != BXMG_OK) return st;
        Run R{H, ctx->stream, 0, 0, 2, 1e-12};
        const Level& L0 = *H->L[0];
        const Level& L1 = *H->L[1];
        HIPCHK(launch_fab_to_rb(R.s, L0.grid(), (const double*)fine->data, fine->d_fboxes.p, H->u64[0]->p, false));
        HIPCHK(launch_restrict_plain<double>(R.s, H->xgrid(0), H->u64[0]->p, H->f64[1]->p));
        HIPCHK(launch_rb_to_fab(R.s, L1.grid(), H->f64[1]->p, (double*)coarse->data, coarse->d_fboxes.p));
        HIPCHK(hipStreamSynchronize(R.s));
    } catch (HipError& e) {
        return fail(BXMG_EDEVICE, std::string("restrict: ") + e.where + ": " + hipGetErrorString(e.e));
    }
    return BXMG_OK;
}

bxmg_status bxmg_prolong_add(bxmg_ctx ctx, bxmg_multifab coarse, bxmg_multifab fine, int32_t order) {
    if (!ctx || !fine || !coarse) return fail(BXMG_EINVAL, "prolong_add: NULL argument");
    if (order != 1 && order != 2) return fail(BXMG_EINVAL, "prolong_add: order must be 1 or 2");
    std::lock_guard<std::mutex> lock(ctx->mu);
    try {
        HIPCHK(hipSetDevice(ctx->device));
        Hier* H;
        bxmg_status st = stage_prepare(ctx, fine, nullptr, nullptr, 1.0, &H);
        if (st != BXMG_OK) return st;
        if (H->L.size() < 2 || !same_boxes(H->L[1]->boxes, coarse->ba->boxes))
            return fail(BXMG_EINVAL, "prolong_add: coarse BoxArray is not the next level of the fine one");
        if ((st = check_solve_mf(coarse, coarse->ba, "coarse")) != BXMG_OK) return st;
        Run R{H, ctx->stream, 0, 0, order, 1e-12};
        const Level& L0 = *H->L[0];
        const Level& L1 = *H->L[1];
        HIPCHK(launch_fab_to_rb(R.s, L0.grid(), (const double*)fine->data, fine->d_fboxes.p, H->u64[0]->p, false));
        HIPCHK(launch_fab_to_rb(R.s, L1.grid(), (const double*)coarse->data, coarse->d_fboxes.p, H->u64[1]->p, false));
        fill<double>(R, 1, H->u64[1]->p, L1.full);
        HIPCHK(launch_prolong<double>(R.s, L0.grid(), L1.d_rb.p, L0.cbox.p, H->u64[1]->p, H->u64[0]->p, order));
        HIPCHK(launch_rb_to_fab(R.s, L0.grid(), H->u64[0]->p, (double*)fine->data, fine->d_fboxes.p));
        HIPCHK(hipStreamSynchronize(R.s));
    } catch (HipError& e) {
        return fail(BXMG_EDEVICE, std::string("prolong_add: ") + e.where + ": " + hipGetErrorString(e.e));
    }
    return BXMG_OK;
}

bxmg_status bxmg_bottom_solve(bxmg_ctx ctx, bxmg_multifab phi, bxmg_multifab rhs, bxmg_multifab beta, double h,
                              double rtol, int32_t* iters) {
    if (!rhs) return fail(BXMG_EINVAL, "bottom_solve: rhs is NULL");
    if (beta) return fail(BXMG_EINVAL, "bottom_solve: variable coefficients are only supported inside a solve");
    if (phi && !bottom_fits(phi->ba->dom))
        return fail(BXMG_EINVAL, "bottom_solve: more than 4096 cells (or 6144 with the ghost layer)");
    if (phi && !covers_domain(phi->ba)) return fail(BXMG_EINVAL, "bottom_solve: the BoxArray must cover its domain");
    std::lock_guard<std::mutex> lock(ctx->mu);
    try {
        HIPCHK(hipSetDevice(ctx->device));
        Hier* H;
        bxmg_status st = stage_prepare(ctx, phi, rhs, nullptr, h, &H);
        if (st != BXMG_OK) return st;
        Run R{H, ctx->stream, 0, 0, 2, rtol};
        const Level& L0 = *H->L[0];
        HIPCHK(launch_fab_to_rb(R.s, L0.grid(), (const double*)rhs->data, rhs->d_fboxes.p, H->f64[0]->p, false));
        HIPCHK(launch_bottom<double>(R.s, H->u64[0]->p, H->f64[0]->p, no_faces<double>(), false, L0.d_rb.p,
                                     (int)L0.boxes.size(), L0.dom.lo, L0.dom.hi, H->per, L0.h, 0.0, rtol, H->iters.p));
        HIPCHK(launch_rb_to_fab(R.s, L0.grid(), H->u64[0]->p, (double*)phi->data, phi->d_fboxes.p));
        int it = 0;
        HIPCHK(hipMemcpyAsync(&it, H->iters.p, sizeof(int), hipMemcpyDeviceToHost, R.s));
        HIPCHK(hipStreamSynchronize(R.s));
        if (iters) *iters = it;
    } catch (HipError& e) {
        return fail(BXMG_EDEVICE, std::string("bottom_solve: ") + e.where + ": " + hipGetErrorString(e.e));
    }
    return BXMG_OK;
}

}  // extern "C"
