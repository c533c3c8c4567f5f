// Batch engine of libbxmg: many independent problems in flight together.
//
// All problems share one arena per storage kind (u, f and beta in FP64, and
// in FP32 for the mixed form).  A problem owns one contiguous element range
// of that arena, laid out level by level in the colour-split format of the
// single-problem driver, so its level data sit at the same offsets in every
// kind.  Everything that depends only on a problem's geometry (hierarchy,
// box layouts, ghost lists, tiles) is built once per geometry as a GeoPlan
// whose offsets are relative to the problem start, and shared by every
// problem of that shape; a problem itself is an arena offset and a slot.
//
// For each level index l the batch concatenates the boxes of every running
// problem that has a level l, and the stage kernels run once per level over
// all of them (boxes carry their problem slot and grid spacing).  The
// trailing single-box levels of every problem run in one launch of the fused
// coarse cycle, one workgroup per problem.  A cycle's residual norms are
// reduced per problem and a device-side stop test retires the problems that
// are done; later launches skip their boxes.  The whole cycle is captured as
// a hipGraph and replayed until the host looks again.  Admission and
// retirement enqueue their conversions without waiting; a step synchronises
// once.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <deque>

#include "../../include/bxmg.h"
#include "bxmg_host.h"
#include "bxmg_internal.h"

static_assert(kStatusNoConv == BXMG_ENOCONV && kStatusNonFinite == BXMG_ENONFINITE, "status codes");

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over element indices [0, cap).
struct Ranges {
    std::map<long long, long long> free;  // start -> length
    void init(long long cap) {
        free.clear();
        if (cap > 0) free[0] = cap;
    }
    long long take(long long n) {
        if (n <= 0) return 0;
        for (auto it = free.begin(); it != free.end(); ++it)
            if (it->second >= n) {
                const long long s = it->first, len = it->second;
                free.erase(it);
                if (len > n) free[s + n] = len - n;
                return s;
            }
        return -1;
    }
    void give(long long s, long long n) {
        if (n <= 0) return;
        auto it = free.emplace(s, n).first;
        auto nx = std::next(it);
        if (nx != free.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free.erase(nx);
        }
        if (it != free.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free.erase(it);
            }
        }
    }
    long long free_total() const {
        long long t = 0;
        for (auto& r : free) t += r.second;
        return t;
    }
};

// ------------------------------------------------------------------- plans
// One level of a geometry; element offsets relative to the problem start.
struct PlanLevel {
    Box dom;
    double h = 0;
    std::vector<Box> boxes;
    std::vector<RBox> rb;
    long long off = 0, nelem = 0;
    bool push = false;
    std::vector<int> cbox;  // coarse owner (level l+1, local index)
    std::vector<std::array<int, 3>> ecol, edown;
    std::vector<Tile> tcol, tdown;  // tiles of the level alone (box = local index)
    int stage_values = 0;           // prolongation: coarse values a colour tile reads (bound)
    DevBuf<GhostCopy> face[2], full;    // indices relative to the problem start
    DevBuf<GhostCopy> face01;           // level 0: both colours' face ghosts in one list (admission)
    DevBuf<GhostCopy> cface[2], cfull;  // relative to the level start (coarse-cycle levels)
    long long fface[3] = {0, 0, 0};     // face-array offsets (variable coefficient)
};

struct GeoPlan {
    Box dom;
    int per[3] = {0, 0, 0};
    std::vector<PlanLevel> L;
    int cs = -1;  // first level of the fused coarse cycle
    long long len = 0, face_len = 0;
    // level 0 (and 1, for the coefficient setup) of one problem alone
    DevBuf<RBox> rb0, rb1;
    // the caller's level-0 boxes; when level 0 runs merged, views of them
    // into the merged storage serve the conversions, the norm of f and the mean
    std::vector<Box> boxes0;
    bool merged0 = false;
    DevBuf<RBox> vrb0;
    DevBuf<Tile> t0;
    int nt0 = 0;
    std::vector<RBox> view0_h;  // host copies: the boxes of grid0() and its tiles
    std::vector<Tile> t0_h;
    int res0 = 0;
    DevBuf<GhostCopy> full_even0;
    DevBuf<int> cbox0;
    DevBuf<Tile> tface[3];
    int ntface[3] = {0, 0, 0};
    Grid grid0() const {
        return merged0 ? Grid{vrb0.p, t0.p, nt0, 0, nullptr, 0, 0}
                       : Grid{rb0.p, t0.p, nt0, L[0].push ? 1 : 0, nullptr, 0, res0};
    }
    XGrid face_grid(int d) const {
        return XGrid{rb0.p, rb1.p, cbox0.p, tface[d].p, ntface[d], 0, nullptr, 0, 0};
    }
};

// Geometry only (no device work): hierarchy, coarse-cycle start, layout.
// False (with a reason) if the problem cannot run in a batch.
bool plan_geometry(const bxmg_ba_s* ba, double h0, GeoPlan& P, std::string* why) {
    P.dom = ba->dom;
    for (int d = 0; d < 3; ++d) P.per[d] = ba->per[d];
    const std::vector<LevelBoxes> lb = make_hierarchy(ba->dom, ba->boxes);
    if (!bottom_fits(lb.back().dom)) {
        if (why) *why = "bottom level above 4096 cells";
        return false;
    }
    const size_t nl = lb.size();
    P.cs = -1;
    for (size_t l = 1; l < nl; ++l) {
        bool ok = nl - l <= (size_t)kMaxCoarseLevels;
        for (size_t m = l; m < nl && ok; ++m) ok = lb[m].boxes.size() == 1 && lb[m].dom.cells() <= kMaxBottomCells;
        if (ok) { P.cs = (int)l; break; }
    }
    if (P.cs < 0) {
        if (why) *why = "the trailing levels are not single boxes of at most 4096 cells";
        return false;
    }
    P.L.clear();
    P.L.resize(nl);
    P.boxes0 = lb[0].boxes;
    long long off = 0, foff = 0;
    double h = h0;
    for (size_t l = 0; l < nl; ++l) {
        PlanLevel& v = P.L[l];
        v.dom = lb[l].dom;
        v.h = h;
        h *= 2.0;
        v.boxes = execution_boxes(lb[l], l, true);
        v.rb = rb_layout(v.boxes, 1, v.h, &v.nelem);
        v.push = face_neighbours(v.dom, P.per, v.boxes, v.rb);
        v.off = off;
        for (auto& r : v.rb) r.base += off;
        off += v.nelem;
        if (l + 1 < nl) v.cbox = coarse_owner(v.boxes, execution_boxes(lb[l + 1], l + 1));
        v.ecol = colour_extents(v.boxes);
        if (l + 1 < nl) v.edown = coarse_extents(v.boxes, v.dom, -1);
        if (l >= 1)
            for (int d = 0; d < 3; ++d) {
                v.fface[d] = foff;
                foff += (long long)(v.dom.n(0) + (d == 0)) * (v.dom.n(1) + (d == 1)) * (v.dom.n(2) + (d == 2));
            }
    }
    P.len = (off + 63) / 64 * 64;
    P.face_len = (foff + 63) / 64 * 64;
    if (P.len > 0x7fffffffLL) {
        if (why) *why = "level storage beyond 2^31 elements";
        return false;
    }
    return true;
}

// Ghost lists and device structures of a planned geometry.
void plan_device(GeoPlan& P, const bxmg_ctx_s* ctx, bool var) {
    for (size_t l = 0; l < P.L.size(); ++l) {
        PlanLevel& v = P.L[l];
        if ((int)l < P.cs) {
            // batched launches have many problems' tiles: no minimum per problem
            const TileSet tc = level_tiles(v.ecol, ctx->zc, ctx->zc_planes, ctx->ly_cap, 0);
            v.tcol = tc.tiles;
            v.stage_values = prolong_stage_values(tc.sh);
            v.tdown = make_tiles(v.edown, ctx->zc, ctx->ly_cap).tiles;
        }
        const std::vector<Tag> faces = build_tags(v.dom, P.per, v.boxes, 1, true, 2, true);
        const std::vector<GhostCopy> f0 = ghost_list(faces, v.rb, 1), f1 = ghost_list(faces, v.rb, 2);
        const std::vector<GhostCopy> full = ghost_list(build_tags(v.dom, P.per, v.boxes, 1, false, 2, true), v.rb, 3);
        if ((int)l < P.cs) {
            v.face[0].upload(f0);
            v.face[1].upload(f1);
            if (l == 0) {
                std::vector<GhostCopy> both(f0);
                both.insert(both.end(), f1.begin(), f1.end());
                v.face01.upload(both);
            }
        }
        if (l >= 1 && (int)l <= P.cs) v.full.upload(full);
        if ((int)l >= P.cs) {
            auto rel = [&](const std::vector<GhostCopy>& a) {
                std::vector<GhostCopy> o(a);
                for (auto& g : o) {
                    g.dst -= (uint32_t)v.off;
                    g.src = ((g.src & 0x7fffffffu) - (uint32_t)v.off) | (g.src & 0x80000000u);
                }
                return o;
            };
            v.cface[0].upload(rel(f0));
            v.cface[1].upload(rel(f1));
            v.cfull.upload(rel(full));
        }
    }
    const PlanLevel& L0 = P.L[0];
    P.rb0.upload(L0.rb);
    P.rb1.upload(P.L[1].rb);
    P.cbox0.upload(L0.cbox);
    P.res0 = (ctx->res && boxes_fit_res(L0.rb)) ? 1 : 0;
    P.merged0 = L0.boxes.size() != P.boxes0.size();
    if (P.merged0) {
        std::vector<RBox> v;
        for (const Box& b : P.boxes0) {
            RBox r = L0.rb[0];
            for (int d = 0; d < 3; ++d) { r.lo[d] = b.lo[d]; r.hi[d] = b.hi[d]; }
            for (int q = 0; q < 6; ++q) { r.nb[q] = -1; r.shift[q] = 0; }
            v.push_back(r);
        }
        P.vrb0.upload(v);
        P.view0_h = v;
    } else {
        P.view0_h = L0.rb;
    }
    // the problem's own level-0 tiles over the caller's boxes: those over
    // which a lone solve sums the periodic mean (the conversions and the
    // norm of f run over them too)
    const std::vector<Tile> t0 = mean_tiles(colour_extents(P.boxes0)).tiles;
    P.t0.upload(t0);
    P.t0_h = t0;
    P.nt0 = (int)t0.size();
    if (var) {
        P.full_even0.upload(ghost_list(build_tags(L0.dom, P.per, L0.boxes, 1, false, 2, false), L0.rb, 3));
        for (int d = 0; d < 3; ++d) {
            TileSet tf = make_tiles(coarse_extents(L0.boxes, L0.dom, d), ctx->zc);
            P.tface[d].upload(tf.tiles);
            P.ntface[d] = (int)tf.tiles.size();
        }
    }
}

std::string plan_key(const bxmg_ba_s* ba, double h, const bxmg_ctx_s* ctx) {
    std::string k;
    auto put = [&](long long x) { k.append((const char*)&x, sizeof x); };
    for (int d = 0; d < 3; ++d) { put(ba->dom.lo[d]); put(ba->dom.hi[d]); put(ba->per[d]); }
    put(ctx->zc);
    put(ctx->zc_planes);
    put(ctx->res);
    put(ctx->ly_cap);
    long long hb;
    std::memcpy(&hb, &h, sizeof hb);
    put(hb);
    for (auto& b : ba->boxes)
        for (int d = 0; d < 3; ++d) { put(b.lo[d]); put(b.hi[d]); }
    return k;
}

// ------------------------------------------------------------- problems
struct Problem {
    int64_t id = 0;
    int slot = -1;
    bxmg_multifab phi = nullptr;
    bxmg_multifab rhs = nullptr, beta = nullptr;  // read at admission
    std::shared_ptr<GeoPlan> plan;
    long long off = 0, foff = 0;  // arena ranges
    double rel_tol = 0;
    Clock::time_point t_add;
};

// Launch structures of one level index over the running problems.
struct BLevel {
    DevVec<RBox> rb;
    DevVec<Tile> tcol, tdown;
    int ntcol = 0, ntdown = 0;
    DevVec<int> cbox;
    bool push = true;
    bool one_box = true;  // every member problem's level is one box
    bool coarse_self = true;  // ... and its level l + 1 one box of at most kSelfGhostCells cells
    int res = 1;
    int stage_values = 0;  // largest prolongation stage of the member problems' tiles
    DevVec<GhostSet> face[2], fullc;  // face ghosts of l; every ghost of l + 1
    int nface = 0, nfullc = 0;
    long long mface = 0, mfullc = 0;
    DevVec<FaceArrays<double>> fat64;  // by slot
    DevVec<FaceArrays<float>> fat32;
    int flip = 0;
};

struct Done {
    int64_t id;
    bxmg_solve_info info;
};

}  // namespace

struct bxmg_batch_s {
    bxmg_ctx ctx = nullptr;
    bxmg_solve_params P{};
    bool var = false;
    int prec = 0;
    int max_slots = 0;
    size_t budget = 0;
    long long cap = 0, fcap = 0;  // arena elements, face-arena elements
    Ranges ranges, franges;
    DevBuf<double> u64, f64, b64, fa64;
    DevBuf<float> u32, f32, b32, fa32;
    // per slot
    DevBuf<int> active, nactive;
    // per slot: 0 while the problem's iterate is its all-+0.0 guess (the
    // first residual then skips the reads of u)
    DevBuf<int> guess_nz;
    DevBuf<BatchSlot> st;
    DevBuf<double> norms, hist, hist_l2, fn3;
    int* h_active = nullptr;
    BatchSlot* h_st = nullptr;
    double* h_hist = nullptr;  // the device's hist, then hist_l2 (kHist per slot each)
    std::vector<std::unique_ptr<Problem>> slots;
    std::deque<int> free_slots;
    int64_t next_id = 1;
    std::deque<Done> done;
    std::map<std::string, std::shared_ptr<GeoPlan>> plans;
    std::deque<std::string> plan_lru;
    // launch structures of the running set
    bool dirty = true;
    std::vector<int> members;
    DevVec<int> d_members;
    std::vector<BLevel> lev;
    int lmax = 0;
    DevVec<int> tstart, segslot;
    // problems added since the last launch, admitted together by its first launches
    std::vector<int> pending;
    DevVec<Tile> a_tiles;
    DevVec<RBox> a_rb;
    DevVec<ConvSrc> a_src;
    DevVec<int> a_tstart, a_seg, a_slots;
    DevVec<GhostSet> a_sets;
    DevVec<BatchSlot> a_states;
    DevVec<double> a_part;
    // the stopped problems of a step, converted back together
    DevVec<Tile> r_tiles, m_tiles;
    DevVec<RBox> r_rb, m_rb;
    DevVec<RetireBox> r_info, m_info;
    DevVec<int> m_seg;
    int nseg = 0;
    DevVec<double> partials, scratch;
    DevVec<ZeroRange> z0;
    int nz0 = 0;
    long long z0max = 0;
    DevVec<CoarseCycle<double>> cc64;
    DevVec<CoarseCycle<float>> cc32;
    int ncc = 0;
    int cc_lds = 0;  // dynamic LDS of the coarse-cycle launch
    bool cc_all_lds = false;  // every member's coarse levels fit in LDS
    bool use_graph = true;
    int stable = 0;         // launches since the running set last changed
    bool inflight = false;  // cycles launched and not yet collected
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // the batch's own stream (default priority): graphs cannot be captured on
    // the legacy default stream a context may use
    hipStream_t stream = nullptr;
    hipEvent_t caller_ready = nullptr;
    ~bxmg_batch_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (caller_ready) (void)hipEventDestroy(caller_ready);
        if (stream) (void)hipStreamDestroy(stream);
        if (h_active) (void)hipHostFree(h_active);
        if (h_st) (void)hipHostFree(h_st);
        if (h_hist) (void)hipHostFree(h_hist);
    }
};

namespace {

size_t arena_bytes_per_elem(int prec, bool var) {
    size_t e = 16;                // u, f FP64
    if (prec == 1) e += 8;        // u, f FP32
    if (var) e += prec ? 12 : 8;  // beta FP64 (+ FP32)
    return e;
}

// The plan of a geometry (built on first use; the last 64 are kept).
std::shared_ptr<GeoPlan> get_plan(bxmg_batch_s* b, const bxmg_ba_s* ba, double h, std::string* why) {
    const std::string key = plan_key(ba, h, b->ctx);
    auto it = b->plans.find(key);
    if (it != b->plans.end()) return it->second;
    auto P = std::make_shared<GeoPlan>();
    if (!plan_geometry(ba, h, *P, why)) return nullptr;
    plan_device(*P, b->ctx, b->var);
    b->plans[key] = P;
    b->plan_lru.push_back(key);
    if (b->plan_lru.size() > 64) {
        b->plans.erase(b->plan_lru.front());
        b->plan_lru.pop_front();
    }
    return P;
}

template <class T>
FaceArrays<T> face_view(const Problem& p, const T* arena, size_t l) {
    FaceArrays<T> f;
    const PlanLevel& v = p.plan->L[l];
    for (int d = 0; d < 3; ++d) {
        f.c[d] = (l >= 1 && arena) ? arena + p.foff + v.fface[d] : nullptr;
        f.dlo[d] = v.dom.lo[d];
        f.n[d] = v.dom.n(d);
    }
    return f;
}

// face arrays of levels >= 1 from the level-0 cell beta (as the single-problem setup)
template <class T>
void setup_faces(hipStream_t s, const Problem& p, T* beta0, const T* arena) {
    const GeoPlan& P = *p.plan;
    HIPCHK(launch_fill_rb(s, beta0, sizeof(T) == 4, P.full_even0.p, (long long)P.full_even0.n));
    for (size_t l = 1; l < P.L.size(); ++l) {
        const FaceArrays<T> out = face_view<T>(p, arena, l);
        for (int d = 0; d < 3; ++d) {
            T* dst = const_cast<T*>(out.c[d]);
            if (l == 1) HIPCHK(launch_faces_from_cells<T>(s, P.face_grid(d), beta0, d, out, dst));
            else HIPCHK(launch_faces_coarsen<T>(s, face_view<T>(p, arena, l - 1), out, d, dst));
        }
    }
}

template <class T>
CoarseCycle<T> coarse_desc(const bxmg_batch_s* b, const Problem& p, T* u, T* f, const T* faces) {
    const GeoPlan& P = *p.plan;
    CoarseCycle<T> cc;
    std::memset(&cc, 0, sizeof cc);
    cc.nlev = (int)P.L.size() - P.cs;
    cc.nu1 = b->P.nu1;
    cc.nu2 = b->P.nu2;
    cc.prolong = b->P.prolong;
    for (int d = 0; d < 3; ++d) cc.per[d] = P.per[d];
    cc.pid = p.slot;
    cc.rtol = b->P.bottom_rtol;
    cc.iters = nullptr;
    for (int m = 0; m < cc.nlev; ++m) {
        const PlanLevel& v = P.L[P.cs + m];
        CoarseLevel<T>& c = cc.L[m];
        c.box = v.rb[0];
        c.box.base -= v.off;
        c.u = u + p.off + v.off;
        c.f = f + p.off + v.off;
        for (int q = 0; q < 2; ++q) { c.face[q] = v.cface[q].p; c.nface[q] = (long long)v.cface[q].n; }
        c.full = v.cfull.p;
        c.nfull = (long long)v.cfull.n;
        c.nelem = v.nelem;
        c.h = v.h;
        c.fa = face_view<T>(p, faces, P.cs + m);
        c.push = v.push ? 1 : 0;
    }
    return cc;
}

// ------------------------------------------------------------- rebuild
void destroy_graph(bxmg_batch_s* b) {
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
}

void rebuild(bxmg_batch_s* b) {
    destroy_graph(b);
    b->members.clear();
    for (int s = 0; s < b->max_slots; ++s)
        if (b->slots[s] && b->h_active[s]) b->members.push_back(s);
    b->d_members.assign(b->members);
    b->lmax = 0;
    b->ncc = 0;
    b->nseg = 0;
    b->dirty = false;
    if (b->members.empty()) return;
    size_t depth = 0;
    for (int s : b->members) {
        depth = std::max(depth, b->slots[s]->plan->L.size());
        b->lmax = std::max(b->lmax, b->slots[s]->plan->cs);
    }
    if (b->lev.size() < depth) b->lev.resize(depth);
    std::vector<std::vector<int>> first(depth, std::vector<int>(b->max_slots, -1));  // first box of slot at level
    std::vector<std::vector<RBox>> rbs(depth);
    for (size_t l = 0; l < depth; ++l)
        for (int s : b->members) {
            const Problem& p = *b->slots[s];
            if (l >= p.plan->L.size()) continue;
            first[l][s] = (int)rbs[l].size();
            for (const RBox& r0 : p.plan->L[l].rb) {
                RBox r = r0;
                r.base += p.off;
                r.pid = s;
                for (int q = 0; q < 6; ++q)
                    if (r.nb[q] >= 0) r.nb[q] += first[l][s];
                rbs[l].push_back(r);
            }
        }
    std::vector<int> tstart{0}, segslot;
    for (size_t l = 0; l < depth; ++l) {
        BLevel& B = b->lev[l];
        B.rb.assign(rbs[l]);
        B.res = (b->ctx->res && boxes_fit_res(rbs[l])) ? 1 : 0;
        B.ntcol = B.ntdown = B.nface = B.nfullc = 0;
        if ((int)l >= b->lmax) continue;
        // tiled problems at l: colour tiles, transfer tiles, ghost sets
        std::vector<Tile> tcol, tdown;
        std::vector<int> cbox_full(rbs[l].size(), -1);
        std::vector<GhostSet> face[2], fullc;
        B.push = true;
        B.one_box = true;
        B.coarse_self = true;
        B.stage_values = 0;
        B.mface = B.mfullc = 0;
        for (int s : b->members) {
            const Problem& p = *b->slots[s];
            if ((int)l >= p.plan->cs) continue;
            const PlanLevel& v = p.plan->L[l];
            const int f0 = first[l][s];
            if (l == 0) segslot.push_back(s);
            for (Tile t : v.tcol) { t.box += f0; tcol.push_back(t); }
            B.stage_values = std::max(B.stage_values, v.stage_values);
            for (Tile t : v.tdown) { t.box += f0; tdown.push_back(t); }
            if (l == 0) tstart.push_back((int)tcol.size());
            for (size_t q = 0; q < v.boxes.size(); ++q) cbox_full[f0 + q] = first[l + 1][s] + v.cbox[q];
            B.push = B.push && v.push;
            B.one_box = B.one_box && v.boxes.size() == 1;
            for (int c = 0; c < 2; ++c) face[c].push_back(GhostSet{v.face[c].p, (long long)v.face[c].n, p.off, s, 0});
            B.mface = std::max(B.mface, (long long)std::max(v.face[0].n, v.face[1].n));
            const PlanLevel& w = p.plan->L[l + 1];
            B.coarse_self = B.coarse_self && w.boxes.size() == 1 && w.dom.cells() <= kSelfGhostCells;
            fullc.push_back(GhostSet{w.full.p, (long long)w.full.n, p.off, s, 0});
            B.mfullc = std::max(B.mfullc, (long long)w.full.n);
        }
        B.tcol.assign(tcol);
        B.ntcol = (int)tcol.size();
        B.tdown.assign(tdown);
        B.ntdown = (int)tdown.size();
        B.cbox.assign(cbox_full);
        if (!B.push) {
            for (int c = 0; c < 2; ++c) B.face[c].assign(face[c]);
            B.nface = (int)face[0].size();
        }
        B.fullc.assign(fullc);
        B.nfullc = (int)fullc.size();
    }
    b->tstart.assign(tstart);
    b->segslot.assign(segslot);
    b->nseg = (int)segslot.size();
    b->partials.reserve(3 * (size_t)std::max(1, b->lev[0].ntcol) + 8);
    // level-0 ranges (the FP32 correction starts from zero every cycle)
    std::vector<ZeroRange> z0;
    b->z0max = 0;
    for (int s : b->members) {
        const Problem& p = *b->slots[s];
        const PlanLevel& v = p.plan->L[0];
        z0.push_back(ZeroRange{p.off + v.off, v.nelem, s, 0});
        b->z0max = std::max(b->z0max, v.nelem);
    }
    b->z0.assign(z0);
    b->nz0 = (int)z0.size();
    // coefficient tables by slot
    if (b->var)
        for (size_t l = 1; l < depth; ++l) {
            BLevel& B = b->lev[l];
            if (b->prec == 0) {
                std::vector<FaceArrays<double>> t(b->max_slots);
                std::memset(t.data(), 0, t.size() * sizeof(t[0]));
                for (int s : b->members)
                    if (l < b->slots[s]->plan->L.size()) t[s] = face_view<double>(*b->slots[s], b->fa64.p, l);
                B.fat64.assign(t);
            } else {
                std::vector<FaceArrays<float>> t(b->max_slots);
                std::memset(t.data(), 0, t.size() * sizeof(t[0]));
                for (int s : b->members)
                    if (l < b->slots[s]->plan->L.size()) t[s] = face_view<float>(*b->slots[s], b->fa32.p, l);
                B.fat32.assign(t);
            }
        }
    // fused coarse cycles (dynamic LDS: the largest need of a member)
    b->cc_lds = 0;
    b->cc_all_lds = true;
    if (b->prec == 0) {
        std::vector<CoarseCycle<double>> cc;
        for (int s : b->members) {
            cc.push_back(coarse_desc<double>(b, *b->slots[s], b->u64.p, b->f64.p, b->fa64.p));
            b->cc_lds = std::max(b->cc_lds, coarse_lds_layout<double>(cc.back(), b->ctx->lds_coarse));
            b->cc_all_lds = b->cc_all_lds && cc.back().lds;
        }
        b->cc64.assign(cc);
    } else {
        std::vector<CoarseCycle<float>> cc;
        for (int s : b->members) {
            cc.push_back(coarse_desc<float>(b, *b->slots[s], b->u32.p, b->f32.p, b->fa32.p));
            b->cc_lds = std::max(b->cc_lds, coarse_lds_layout<float>(cc.back(), b->ctx->lds_coarse));
            b->cc_all_lds = b->cc_all_lds && cc.back().lds;
        }
        b->cc32.assign(cc);
    }
    b->ncc = (int)b->members.size();
}

// -------------------------------------------------------------- the cycle
template <class T>
T* arena_u(bxmg_batch_s* b);
template <>
double* arena_u<double>(bxmg_batch_s* b) { return b->u64.p; }
template <>
float* arena_u<float>(bxmg_batch_s* b) { return b->u32.p; }
template <class T>
T* arena_f(bxmg_batch_s* b);
template <>
double* arena_f<double>(bxmg_batch_s* b) { return b->f64.p; }
template <>
float* arena_f<float>(bxmg_batch_s* b) { return b->f32.p; }
template <class T>
const T* arena_beta(bxmg_batch_s* b, size_t l);
template <>
const double* arena_beta<double>(bxmg_batch_s* b, size_t l) { return (b->var && l == 0) ? b->b64.p : nullptr; }
template <>
const float* arena_beta<float>(bxmg_batch_s* b, size_t l) { return (b->var && l == 0) ? b->b32.p : nullptr; }
template <class T>
const FaceArrays<T>* level_fat(bxmg_batch_s* b, size_t l);
template <>
const FaceArrays<double>* level_fat<double>(bxmg_batch_s* b, size_t l) {
    return (b->var && l >= 1) ? b->lev[l].fat64.p() : nullptr;
}
template <>
const FaceArrays<float>* level_fat<float>(bxmg_batch_s* b, size_t l) {
    return (b->var && l >= 1) ? b->lev[l].fat32.p() : nullptr;
}
template <class T>
const CoarseCycle<T>* coarse_descs(bxmg_batch_s* b);
template <>
const CoarseCycle<double>* coarse_descs<double>(bxmg_batch_s* b) { return b->cc64.p(); }
template <>
const CoarseCycle<float>* coarse_descs<float>(bxmg_batch_s* b) { return b->cc32.p(); }

Grid level_grid(bxmg_batch_s* b, size_t l) {
    BLevel& B = b->lev[l];
    Grid g{B.rb.p(), B.tcol.p(), B.ntcol, B.push ? (B.one_box ? 2 : 1) : 0, b->active.p, B.flip, B.res};
    B.flip ^= 1;
    return g;
}

XGrid level_xgrid(bxmg_batch_s* b, size_t l) {
    BLevel& B = b->lev[l];
    XGrid x{B.rb.p(), b->lev[l + 1].rb.p(), B.cbox.p(), B.tdown.p(), B.ntdown, B.push ? 1 : 0,
            b->active.p, B.flip, (B.res && b->lev[l + 1].res) ? 1 : 0};
    B.flip ^= 1;
    return x;
}

template <class T>
void b_smooth(bxmg_batch_s* b, hipStream_t s, size_t l, int nsweeps) {
    BLevel& B = b->lev[l];
    T* u = arena_u<T>(b);
    for (int k = 0; k < nsweeps; ++k)
        for (int c = 0; c < 2; ++c) {
            if (!B.push)
                HIPCHK(launch_fill_sets(s, u, sizeof(T) == 4, B.face[c ^ 1].p(), B.nface, B.mface, b->active.p));
            HIPCHK(launch_gs<T>(s, level_grid(b, l), u, arena_f<T>(b), arena_beta<T>(b, l), level_fat<T>(b, l), c));
        }
}

template <class T>
void b_vcycle(bxmg_batch_s* b, hipStream_t s) {
    T* u = arena_u<T>(b);
    T* f = arena_f<T>(b);
    const bool f32 = sizeof(T) == 4;
    for (int l = 0; l < b->lmax; ++l) {
        BLevel& B = b->lev[l];
        b_smooth<T>(b, s, l, b->P.nu1);
        if (!B.push) {
            HIPCHK(launch_fill_sets(s, u, f32, B.face[0].p(), B.nface, B.mface, b->active.p));
            HIPCHK(launch_fill_sets(s, u, f32, B.face[1].p(), B.nface, B.mface, b->active.p));
        }
        // the coarse correction starts from zero: zeroed by the same launch
        // (cells and the face ghosts mirroring them)
        HIPCHK(launch_resid_restrict<T>(s, level_xgrid(b, l), u, f, arena_beta<T>(b, l), level_fat<T>(b, l), f, u));
    }
    HIPCHK(launch_coarse_cycle<T>(s, coarse_descs<T>(b), b->ncc, b->active.p, b->var, b->cc_lds, b->cc_all_lds));
    for (int l = b->lmax - 1; l >= 0; --l) {
        BLevel& B = b->lev[l];
        // small one-box coarse levels: the staged prolongation reads the
        // cells their ghosts mirror, so no ghost refresh before it
        const Grid g = level_grid(b, l);
        const bool self = B.coarse_self && prolong_staged(g.push, b->P.nu2 > 0, B.stage_values);
        if (!self) HIPCHK(launch_fill_sets(s, u, f32, B.fullc.p(), B.nfullc, B.mfullc, b->active.p));
        HIPCHK(launch_prolong<T>(s, g, b->lev[l + 1].rb.p(), B.cbox.p(), u, u, b->P.prolong, b->P.nu2 > 0,
                                 B.stage_values, self));
        b_smooth<T>(b, s, l, b->P.nu2);
    }
}

// One batch cycle: FP64 residual and per-problem norms, the stop test, and
// the V-cycle (FP64, or FP32 correction added to the FP64 solution).
void enqueue_cycle(bxmg_batch_s* b, hipStream_t s) {
    const double* beta0 = b->var ? b->b64.p : nullptr;
    if (b->prec == 0)
        HIPCHK(launch_resid<double, double>(s, level_grid(b, 0), b->u64.p, b->f64.p, beta0, nullptr, (double*)nullptr,
                                            b->partials.p(), false, b->guess_nz.p));
    else
        HIPCHK(launch_resid<double, float>(s, level_grid(b, 0), b->u64.p, b->f64.p, beta0, nullptr, b->f32.p,
                                           b->partials.p(), false, b->guess_nz.p));
    HIPCHK(launch_norm_seg(s, b->partials.p(), b->tstart.p(), b->segslot.p(), b->nseg, b->active.p, b->norms.p));
    HIPCHK(launch_batch_check(s, b->d_members.p(), (int)b->members.size(), b->norms.p, b->st.p, b->active.p,
                              b->hist.p, b->hist_l2.p, b->nactive.p, b->guess_nz.p));
    if (b->prec == 0) {
        b_vcycle<double>(b, s);
    } else {
        HIPCHK(launch_zero_ranges<float>(s, b->u32.p, b->z0.p(), b->nz0, b->z0max, b->active.p));
        b_vcycle<float>(b, s);
        HIPCHK(launch_add_f32(s, level_grid(b, 0), b->u64.p, b->u32.p));
    }
}

// -------------------------------------------------------- finish / release
void release_problem(bxmg_batch_s* b, int s) {
    Problem& p = *b->slots[s];
    b->ranges.give(p.off, p.plan->len);
    if (b->var) b->franges.give(p.foff, p.plan->face_len);
    b->slots[s].reset();
    b->h_active[s] = 0;
    b->free_slots.push_back(s);
}

// Enqueues the copy of stopped problems' histories: per problem for a few,
// else the whole history arrays in two copies (one per array, instead of two
// per problem).
constexpr size_t kBulkHistory = 16;
void copy_histories(bxmg_batch_s* b, const std::vector<int>& stopped) {
    hipStream_t st = b->stream;
    const size_t all = (size_t)b->max_slots * kHist;
    if (stopped.size() > kBulkHistory) {
        HIPCHK(hipMemcpyAsync(b->h_hist, b->hist.p, all * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(b->h_hist + all, b->hist_l2.p, all * sizeof(double), hipMemcpyDeviceToHost, st));
        return;
    }
    for (int s : stopped) {
        HIPCHK(hipMemcpyAsync(b->h_hist + (size_t)s * kHist, b->hist.p + (size_t)s * kHist, kHist * sizeof(double),
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(b->h_hist + all + (size_t)s * kHist, b->hist_l2.p + (size_t)s * kHist,
                              kHist * sizeof(double), hipMemcpyDeviceToHost, st));
    }
}

// Enqueues the conversion of stopped problems' solutions into their phi:
// the zero solution of a zero right-hand side per problem, then for all of
// them at once the mean subtraction of the fully periodic ones and the
// conversion into the caller layout (a few launches for any number).
void append_retire(const Problem& p, int seg, std::vector<Tile>& tiles, std::vector<RBox>& rbs,
                   std::vector<RetireBox>& info) {
    const GeoPlan& P = *p.plan;
    const int box0 = (int)rbs.size(), t0 = (int)tiles.size();
    for (size_t k = 0; k < P.view0_h.size(); ++k) {
        RBox r = P.view0_h[k];
        r.base += p.off;
        rbs.push_back(r);
        RetireBox R{};
        R.fab = (double*)p.phi->data;
        R.f = p.phi->fboxes[k];
        R.tstart = t0;
        R.nt = (int)P.t0_h.size();
        R.seg = seg;
        info.push_back(R);
    }
    for (Tile t : P.t0_h) {
        t.box += box0;
        tiles.push_back(t);
    }
}

void retire_convert(bxmg_batch_s* b, const std::vector<int>& conv) {
    if (conv.empty()) return;
    hipStream_t st = b->stream;
    std::vector<Tile> tiles, mtiles;
    std::vector<RBox> rbs, mrbs;
    std::vector<RetireBox> info, minfo;
    std::vector<int> mseg{0};
    for (int s : conv) {
        const Problem& p = *b->slots[s];
        const GeoPlan& P = *p.plan;
        if (b->h_st[s].fnorm == 0.0 && b->h_st[s].status == 0)  // f == 0: the solution is u = 0
            HIPCHK(launch_zero<double>(st, b->u64.p + p.off + P.L[0].off, P.L[0].nelem));
        append_retire(p, 0, tiles, rbs, info);
        if (P.per[0] && P.per[1] && P.per[2]) {
            append_retire(p, (int)mseg.size() - 1, mtiles, mrbs, minfo);
            mseg.push_back((int)mtiles.size());
        }
    }
    if (!mtiles.empty()) {
        b->m_tiles.assign(mtiles);
        b->m_rb.assign(mrbs);
        b->m_info.assign(minfo);
        b->m_seg.assign(mseg);
        b->scratch.reserve(3 * (mtiles.size() + mseg.size()) + 8);
        const Grid mg{b->m_rb.p(), b->m_tiles.p(), (int)mtiles.size(), 0, nullptr, 0, 0};
        HIPCHK(launch_mean_sub_many(st, mg, b->m_info.p(), b->m_seg.p(), (int)mseg.size() - 1, b->u64.p,
                                    b->scratch.p()));
    }
    b->r_tiles.assign(tiles);
    b->r_rb.assign(rbs);
    b->r_info.assign(info);
    const Grid g{b->r_rb.p(), b->r_tiles.p(), (int)tiles.size(), 0, nullptr, 0, 0};
    HIPCHK(launch_rb_to_fab_many(st, g, b->u64.p, b->r_info.p()));
}

// After the stream drained: the result record, then the slot and ranges go back.
void retire_finish(bxmg_batch_s* b, int s) {
    const Problem& p = *b->slots[s];
    const BatchSlot S = b->h_st[s];
    Done d;
    d.id = p.id;
    std::memset(&d.info, 0, sizeof d.info);
    d.info.status = S.status;
    d.info.cycles = S.cycles;
    d.info.levels = (int)p.plan->L.size();
    d.info.nhist = std::min(S.nhist, kHist);
    d.info.f_inf = (S.status == kStatusNonFinite && S.nhist == 0) ? NAN : S.fnorm;
    const double* h = b->h_hist + (size_t)s * kHist;
    const double* h2 = b->h_hist + (size_t)b->max_slots * kHist + (size_t)s * kHist;
    for (int k = 0; k < d.info.nhist; ++k) {
        d.info.hist[k] = h[k];
        d.info.hist_l2[k] = h2[k];
    }
    if (d.info.nhist > 0) {
        d.info.rel_resid_inf = d.info.hist[d.info.nhist - 1];
        d.info.resid_l2 = d.info.hist_l2[d.info.nhist - 1];
    }
    d.info.seconds = std::chrono::duration<double>(Clock::now() - p.t_add).count();
    b->done.push_back(d);
    release_problem(b, s);
}

}  // namespace

// ================================================================== C ABI
extern "C" {

bxmg_status bxmg_batch_create(bxmg_ctx ctx, size_t hbm_budget_bytes, int32_t max_problems, int32_t var,
                              const bxmg_solve_params* params, bxmg_batch* out) {
    if (!ctx || !out) return fail(BXMG_EINVAL, "batch_create: NULL argument");
    if (max_problems < 1 || max_problems > 4096) return fail(BXMG_EINVAL, "batch_create: max_problems out of [1, 4096]");
    auto b = std::make_unique<bxmg_batch_s>();
    b->ctx = ctx;
    if (params) b->P = *params;
    else bxmg_solve_params_default(&b->P);
    if (b->P.nu1 < 0 || b->P.nu2 < 0 || b->P.max_cycles < 0 || (b->P.precision != 0 && b->P.precision != 1) ||
        (b->P.prolong != 1 && b->P.prolong != 2))
        return fail(BXMG_EINVAL, "batch_create: bad parameters");
    if (b->P.krylov != 0) return fail(BXMG_EINVAL, "batch_create: batches run V-cycle iterations only (krylov = 0)");
    if (b->P.alpha != 0.0) return fail(BXMG_EINVAL, "batch_create: batches solve the Poisson operator (alpha = 0)");
    b->var = var != 0;
    b->prec = b->P.precision;
    b->max_slots = max_problems;
    b->budget = hbm_budget_bytes;
    // coefficient faces of levels >= 1 take about 3/7 of a level-0 array
    const size_t per = arena_bytes_per_elem(b->prec, b->var);
    const size_t fes = b->var ? (b->prec ? 4 : 8) : 0;
    const double face_share = b->var ? (double)fes * 0.45 / (double)(per + fes * 0.45) : 0.0;
    const size_t face_bytes = (size_t)(face_share * (double)hbm_budget_bytes);
    long long cap = (long long)((hbm_budget_bytes - face_bytes) / per);
    cap = std::min<long long>(cap, 0x7fffffffLL) / 64 * 64;
    if (cap < 64) return fail(BXMG_EINVAL, "batch_create: budget too small");
    b->cap = cap;
    b->fcap = b->var ? (long long)(face_bytes / fes) / 64 * 64 : 0;
    std::lock_guard<std::mutex> lock(ctx->mu);
    try {
        HIPCHK(hipSetDevice(ctx->device));
        HIPCHK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&b->caller_ready, hipEventDisableTiming));
        b->u64.alloc(cap);
        b->f64.alloc(cap);
        if (b->prec == 1) { b->u32.alloc(cap); b->f32.alloc(cap); }
        if (b->var) {
            b->b64.alloc(cap);
            if (b->prec == 1) { b->b32.alloc(cap); b->fa32.alloc(std::max<long long>(b->fcap, 64)); }
            else b->fa64.alloc(std::max<long long>(b->fcap, 64));
        }
        b->active.alloc(max_problems);
        b->guess_nz.alloc(max_problems);
        HIPCHK(hipMemset(b->active.p, 0, max_problems * sizeof(int)));
        b->nactive.alloc(1);
        b->st.alloc(max_problems);
        b->norms.alloc(3 * (size_t)max_problems);
        b->fn3.alloc(3 * (size_t)max_problems);
        b->hist.alloc((size_t)max_problems * kHist);
        b->hist_l2.alloc((size_t)max_problems * kHist);
        HIPCHK(hipHostMalloc((void**)&b->h_active, max_problems * sizeof(int)));
        HIPCHK(hipHostMalloc((void**)&b->h_st, max_problems * sizeof(BatchSlot)));
        HIPCHK(hipHostMalloc((void**)&b->h_hist, (size_t)max_problems * 2 * kHist * sizeof(double)));
        std::memset(b->h_active, 0, max_problems * sizeof(int));
    } catch (HipError& e) {
        return fail(e.e == hipErrorOutOfMemory ? BXMG_ENOMEM : BXMG_EDEVICE,
                    std::string("batch_create: ") + hipGetErrorString(e.e));
    }
    b->ranges.init(cap);
    b->franges.init(b->fcap);
    b->slots.resize(max_problems);
    for (int s = 0; s < max_problems; ++s) b->free_slots.push_back(s);
    *out = b.release();
    return BXMG_OK;
}

void bxmg_batch_destroy(bxmg_batch b) {
    if (!b) return;
    std::lock_guard<std::mutex> lock(b->ctx->mu);
    (void)hipSetDevice(b->ctx->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    delete b;
}

size_t bxmg_batch_footprint(bxmg_batch b, bxmg_boxarray ba) {
    if (!b || !ba) return 0;
    GeoPlan P;
    try {
        if (!plan_geometry(ba, 1.0, P, nullptr)) return 0;
    } catch (std::exception&) {
        return 0;
    }
    return (size_t)P.len * arena_bytes_per_elem(b->prec, b->var) +
           (b->var ? (size_t)P.face_len * (b->prec ? 4 : 8) : 0);
}

bxmg_status bxmg_batch_add(bxmg_batch b, bxmg_multifab phi, bxmg_multifab rhs, bxmg_multifab beta, double rel_tol,
                           int64_t* id) {
    if (!b || !phi || !rhs || !id) return fail(BXMG_EINVAL, "batch_add: NULL argument");
    if ((beta != nullptr) != b->var)
        return fail(BXMG_EINVAL, b->var ? "batch_add: this batch needs beta" : "batch_add: this batch takes no beta");
    const bxmg_ba_s* ba = phi->ba;
    bxmg_status st;
    if ((st = check_solve_mf(phi, ba, "phi")) != BXMG_OK) return st;
    if ((st = check_solve_mf(rhs, ba, "rhs")) != BXMG_OK) return st;
    if (beta && (st = check_solve_mf(beta, ba, "beta")) != BXMG_OK) return st;
    if (!covers_domain(ba)) return fail(BXMG_EINVAL, "batch_add: the BoxArray must cover its domain");
    if (phi->ctx != b->ctx) return fail(BXMG_EINVAL, "batch_add: phi belongs to another context");
    std::lock_guard<std::mutex> lock(b->ctx->mu);
    if (b->inflight) return fail(BXMG_EINVAL, "batch_add: collect the launched cycles first");
    const double h = (b->P.dx > 0) ? b->P.dx : 1.0 / ba->dom.n(0);
    try {
        HIPCHK(hipSetDevice(b->ctx->device));
        std::string why;
        std::shared_ptr<GeoPlan> plan;
        try {
            plan = get_plan(b, ba, h, &why);
        } catch (std::exception& e) {
            return fail(BXMG_EINVAL, std::string("batch_add: ") + e.what());
        }
        if (!plan) return fail(BXMG_EINVAL, "batch_add: " + why);
        const GeoPlan& P = *plan;
        if (P.len > b->cap || (b->var && P.face_len > b->fcap))
            return fail(BXMG_EINVAL, "batch_add: the problem is larger than the whole arena");
        if (b->free_slots.empty()) return fail(BXMG_EBUSY, "batch_add: every slot is taken");
        const long long base = b->ranges.take(P.len);
        if (base < 0) return fail(BXMG_EBUSY, "batch_add: the arena has no free range of this size");
        long long fbase = 0;
        if (b->var) {
            fbase = b->franges.take(P.face_len);
            if (fbase < 0) {
                b->ranges.give(base, P.len);
                return fail(BXMG_EBUSY, "batch_add: coefficient storage is full");
            }
        }
        const int slot = b->free_slots.front();
        b->free_slots.pop_front();
        auto p = std::make_unique<Problem>();
        p->slot = slot;
        p->id = b->next_id++;
        p->phi = phi;
        p->rhs = rhs;
        p->beta = beta;
        p->plan = plan;
        p->off = base;
        p->foff = fbase;
        p->rel_tol = rel_tol > 0 ? rel_tol : b->P.rel_tol;
        p->t_add = Clock::now();
        b->slots[slot] = std::move(p);
        b->h_active[slot] = 1;  // until the device says otherwise
        b->dirty = true;
        *id = b->slots[slot]->id;
        // the slot state; conversions and the admission decision run with
        // the other problems added before the next launch (admit_pending)
        BatchSlot S{};
        S.rel_tol = b->slots[slot]->rel_tol;
        S.abs_tol = b->P.abs_tol;
        S.max_cycles = b->P.max_cycles;
        S.fixed_cycles = b->P.fixed_cycles;
        b->h_st[slot] = S;
        b->pending.push_back(slot);
    } catch (HipError& e) {
        return fail(e.e == hipErrorOutOfMemory ? BXMG_ENOMEM : BXMG_EDEVICE,
                    std::string("batch_add: ") + e.where + ": " + hipGetErrorString(e.e));
    }
    return BXMG_OK;
}

// Admission of every problem added since the last launch, after the work
// the caller queued on the context's stream so far: the initial guesses and
// right-hand sides of all of them in one conversion launch (with the norms of
// f per tile), their face ghosts in one fill, the norms of f reduced per
// problem, coefficient setup (variable beta, per problem), and the decision
// of every slot in one launch.  Six launches for any number of problems
// (plus the coefficient setup), instead of several per problem.
void admit_pending(bxmg_batch_s* b, hipStream_t s) {
    if (b->pending.empty()) return;
    HIPCHK(hipEventRecord(b->caller_ready, b->ctx->stream));
    HIPCHK(hipStreamWaitEvent(s, b->caller_ready, 0));
    std::vector<Tile> tiles;
    std::vector<RBox> rbs;
    std::vector<ConvSrc> srcs;
    std::vector<int> tstart{0}, seg;
    std::vector<GhostSet> sets;
    std::vector<BatchSlot> states;
    long long max_ghosts = 0;
    for (int slot : b->pending) {
        const Problem& q = *b->slots[slot];
        const GeoPlan& P = *q.plan;
        const int box0 = (int)rbs.size();
        for (size_t k = 0; k < P.view0_h.size(); ++k) {
            RBox r = P.view0_h[k];
            r.base += q.off;
            rbs.push_back(r);
            ConvSrc c;
            c.phi = (const double*)q.phi->data;
            c.rhs = (const double*)q.rhs->data;
            c.fphi = q.phi->fboxes[k];
            c.frhs = q.rhs->fboxes[k];
            c.slot = slot;
            srcs.push_back(c);
        }
        for (Tile t : P.t0_h) {
            t.box += box0;
            tiles.push_back(t);
        }
        tstart.push_back((int)tiles.size());
        seg.push_back(slot);
        const DevBuf<GhostCopy>& fl = P.L[0].face01;
        sets.push_back(GhostSet{fl.p, (long long)fl.n, q.off, slot, 0});
        max_ghosts = std::max(max_ghosts, (long long)fl.n);
        states.push_back(b->h_st[slot]);
    }
    b->a_tiles.assign(tiles);
    b->a_rb.assign(rbs);
    b->a_src.assign(srcs);
    b->a_tstart.assign(tstart);
    b->a_seg.assign(seg);
    b->a_slots.assign(b->pending);
    b->a_sets.assign(sets);
    b->a_states.assign(states);
    b->a_part.reserve(3 * tiles.size() + 8);
    const Grid g{b->a_rb.p(), b->a_tiles.p(), (int)tiles.size(), 0, nullptr, 0, 0};
    HIPCHK(launch_set_slots(s, b->a_slots.p(), (int)b->pending.size(), b->guess_nz.p, 0));
    HIPCHK(launch_admit_convert(s, g, b->a_src.p(), b->u64.p, b->f64.p, b->a_part.p(), b->guess_nz.p));
    // ghosts of the converted guesses (later producers keep them current)
    HIPCHK(launch_fill_sets(s, b->u64.p, false, b->a_sets.p(), (int)sets.size(), max_ghosts, nullptr));
    HIPCHK(launch_norm_seg(s, b->a_part.p(), b->a_tstart.p(), b->a_seg.p(), (int)seg.size(), nullptr, b->fn3.p));
    if (b->var) {
        for (int slot : b->pending) {
            const Problem& q = *b->slots[slot];
            const GeoPlan& P = *q.plan;
            const Grid g0 = P.grid0();
            double* bt = b->b64.p + q.off;
            HIPCHK(launch_fab_to_rb(s, g0, (const double*)q.beta->data, q.beta->d_fboxes.p, bt, false));
            if (b->prec == 0) {
                setup_faces<double>(s, q, bt, b->fa64.p);
            } else {
                HIPCHK(launch_fill_rb(s, bt, false, P.full_even0.p, (long long)P.full_even0.n));
                HIPCHK(launch_cast_f32(s, bt + P.L[0].off, b->b32.p + q.off + P.L[0].off, P.L[0].nelem));
                setup_faces<float>(s, q, b->b32.p + q.off, b->fa32.p);
            }
        }
    }
    HIPCHK(launch_batch_admit_many(s, b->fn3.p, b->a_states.p(), b->a_slots.p(), (int)b->pending.size(), b->st.p,
                                   b->active.p));
    b->pending.clear();
}

static bxmg_status batch_launch(bxmg_batch b, int32_t ncycles) {
    if (ncycles < 1) return fail(BXMG_EINVAL, "batch_launch: ncycles < 1");
    if (b->inflight) return fail(BXMG_EBUSY, "batch_launch: the cycles launched before are not collected");
    hipStream_t s = b->stream;
    try {
        HIPCHK(hipSetDevice(b->ctx->device));
        admit_pending(b, s);
        if (b->dirty) {
            rebuild(b);
            b->stable = 0;
        }
        if (!b->members.empty()) {
            // capture once the running set has stayed the same for a launch:
            // while problems come and go every step, stage-by-stage launches
            // cost less than a capture per step
            if (b->use_graph && !b->exec && b->stable >= 1) {
                HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                try {
                    enqueue_cycle(b, s);
                } catch (HipError&) {
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(s, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                HIPCHK(hipStreamEndCapture(s, &b->graph));
                HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
            }
            for (int c = 0; c < ncycles; ++c) {
                if (b->exec) HIPCHK(hipGraphLaunch(b->exec, s));
                else enqueue_cycle(b, s);
            }
            ++b->stable;
        }
        HIPCHK(hipMemcpyAsync(b->h_active, b->active.p, b->max_slots * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(b->h_st, b->st.p, b->max_slots * sizeof(BatchSlot), hipMemcpyDeviceToHost, s));
        b->inflight = true;
    } catch (HipError& e) {
        return fail(BXMG_EDEVICE, std::string("batch_launch: ") + e.where + ": " + hipGetErrorString(e.e));
    }
    return BXMG_OK;
}

static bxmg_status batch_collect(bxmg_batch b, int32_t* nrunning) {
    hipStream_t s = b->stream;
    try {
        HIPCHK(hipSetDevice(b->ctx->device));
        if (b->inflight) {
            HIPCHK(hipStreamSynchronize(s));
            b->inflight = false;
            std::vector<int> stopped;
            for (int m = 0; m < b->max_slots; ++m)
                if (b->slots[m] && !b->h_active[m]) stopped.push_back(m);
            if (!stopped.empty()) {
                copy_histories(b, stopped);
                // a right-hand side that was not finite leaves phi untouched
                std::vector<int> conv;
                for (int m : stopped)
                    if (!(b->h_st[m].status == kStatusNonFinite && b->h_st[m].nhist == 0)) conv.push_back(m);
                retire_convert(b, conv);
                HIPCHK(hipStreamSynchronize(s));
                for (int m : stopped) retire_finish(b, m);
                // retired problems cost only idle blocks; the launch lists are
                // rebuilt when problems join (add marks them) or once a
                // quarter of the running set has left
                int left = 0;
                for (int m : b->members)
                    if (!b->slots[m]) ++left;
                if (4 * left > (int)b->members.size()) b->dirty = true;
            }
        }
    } catch (HipError& e) {
        b->inflight = false;
        return fail(BXMG_EDEVICE, std::string("batch_collect: ") + e.where + ": " + hipGetErrorString(e.e));
    }
    if (nrunning) {
        int n = 0;
        for (int m = 0; m < b->max_slots; ++m)
            if (b->slots[m] && b->h_active[m]) ++n;
        *nrunning = n;
    }
    return BXMG_OK;
}

bxmg_status bxmg_batch_step(bxmg_batch b, int32_t ncycles, int32_t* nrunning) {
    if (!b) return fail(BXMG_EINVAL, "batch_step: NULL batch");
    std::lock_guard<std::mutex> lock(b->ctx->mu);
    const bxmg_status st = batch_launch(b, ncycles);
    if (st != BXMG_OK) return st;
    return batch_collect(b, nrunning);
}

bxmg_status bxmg_batch_launch(bxmg_batch b, int32_t ncycles) {
    if (!b) return fail(BXMG_EINVAL, "batch_launch: NULL batch");
    std::lock_guard<std::mutex> lock(b->ctx->mu);
    return batch_launch(b, ncycles);
}

bxmg_status bxmg_batch_collect(bxmg_batch b, int32_t* nrunning) {
    if (!b) return fail(BXMG_EINVAL, "batch_collect: NULL batch");
    std::lock_guard<std::mutex> lock(b->ctx->mu);
    return batch_collect(b, nrunning);
}

bxmg_status bxmg_batch_poll(bxmg_batch b, int32_t max, int64_t* ids, bxmg_solve_info* infos, int32_t* ndone) {
    if (!b || !ndone || (max > 0 && (!ids || !infos))) return fail(BXMG_EINVAL, "batch_poll: NULL argument");
    std::lock_guard<std::mutex> lock(b->ctx->mu);
    int n = 0;
    while (n < max && !b->done.empty()) {
        ids[n] = b->done.front().id;
        infos[n] = b->done.front().info;
        b->done.pop_front();
        ++n;
    }
    *ndone = n;
    return BXMG_OK;
}

bxmg_status bxmg_batch_remove(bxmg_batch b, int64_t id) {
    if (!b) return fail(BXMG_EINVAL, "batch_remove: NULL batch");
    std::lock_guard<std::mutex> lock(b->ctx->mu);
    for (auto it = b->done.begin(); it != b->done.end(); ++it)
        if (it->id == id) {
            b->done.erase(it);
            return BXMG_OK;
        }
    if (b->inflight) return fail(BXMG_EINVAL, "batch_remove: collect the launched cycles first");
    for (int s = 0; s < b->max_slots; ++s)
        if (b->slots[s] && b->slots[s]->id == id) {
            auto pend = std::find(b->pending.begin(), b->pending.end(), s);
            if (pend != b->pending.end()) {  // not admitted on the device yet
                b->pending.erase(pend);
                release_problem(b, s);
                b->dirty = true;
                return BXMG_OK;
            }
            try {
                HIPCHK(hipSetDevice(b->ctx->device));
                HIPCHK(hipStreamSynchronize(b->stream));
                const int zero = 0;
                HIPCHK(hipMemcpy(b->active.p + s, &zero, sizeof zero, hipMemcpyHostToDevice));
            } catch (HipError& e) {
                return fail(BXMG_EDEVICE, std::string("batch_remove: ") + hipGetErrorString(e.e));
            }
            release_problem(b, s);
            b->dirty = true;
            return BXMG_OK;
        }
    return fail(BXMG_EINVAL, "batch_remove: unknown id");
}

bxmg_status bxmg_batch_stats(bxmg_batch b, size_t* bytes_used, size_t* bytes_budget, int32_t* nrunning,
                             int32_t* nqueued) {
    if (!b) return fail(BXMG_EINVAL, "batch_stats: NULL batch");
    std::lock_guard<std::mutex> lock(b->ctx->mu);
    const size_t per = arena_bytes_per_elem(b->prec, b->var);
    if (bytes_used)
        *bytes_used = (size_t)(b->cap - b->ranges.free_total()) * per +
                      (b->var ? (size_t)(b->fcap - b->franges.free_total()) * (b->prec ? 4 : 8) : 0);
    if (bytes_budget) *bytes_budget = b->budget;
    if (nrunning) {
        int n = 0;
        for (int s = 0; s < b->max_slots; ++s)
            if (b->slots[s] && b->h_active[s]) ++n;
        *nrunning = n;
    }
    if (nqueued) *nqueued = (int32_t)b->done.size();
    return BXMG_OK;
}

bxmg_status bxmg_batch_set(bxmg_batch b, int32_t param, int32_t value) {
    if (!b) return fail(BXMG_EINVAL, "batch_set: NULL batch");
    std::lock_guard<std::mutex> lock(b->ctx->mu);
    if (param != 0 || (value != 0 && value != 1)) return fail(BXMG_EINVAL, "batch_set: unknown parameter or value");
    if (b->inflight) return fail(BXMG_EINVAL, "batch_set: collect the launched cycles first");
    b->use_graph = value != 0;
    destroy_graph(b);
    return BXMG_OK;
}

}  // extern "C"
