// Batch engine of libbxmg: many independent problems in flight together.
//
// All problems share one arena per storage kind (u, f and beta in FP64, and
// in FP32 for the mixed form).  A problem owns one contiguous element range
// of that arena, laid out level by level in the colour-split format of the
// single-problem driver, so its level data sit at the same offsets in every
// kind.  For each level index l the batch concatenates the boxes of every
// running problem that has a level l, and the stage kernels run once per
// level over all of them (boxes carry their problem slot and grid spacing).
// The trailing single-box levels of every problem run in one launch of the
// fused coarse cycle, one workgroup per problem.  A cycle's residual norms
// are reduced per problem and a device-side stop test retires the problems
// that are done; later launches skip their boxes.  The whole cycle is
// captured as a hipGraph and replayed until the host looks again.
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
};

// One level of one problem; RBox bases are absolute arena offsets, face
// neighbours index the problem's own box list of the level.
struct PLevel {
    Box dom;
    double h = 0;
    std::vector<Box> boxes;
    std::vector<RBox> rb;
    long long off = 0, nelem = 0;  // absolute element range of the level
    bool push = false;
    std::vector<GhostCopy> face[2], full;  // absolute element indices
    std::vector<int> cbox;                 // coarse owner (level l+1, local index)
};

template <class T>
struct PFaces {
    DevBuf<T> c[3];
    FaceArrays<T> view{};
};

// Device copies of a level's coarse-cycle ghost lists, indices relative to
// the level's first element.
struct CList {
    DevBuf<GhostCopy> face[2], full;
};

struct Problem {
    int64_t id = 0;
    int slot = -1;
    bxmg_multifab phi = nullptr, rhs = nullptr, beta = nullptr;
    Box dom;
    int per[3] = {0, 0, 0};
    std::vector<PLevel> L;
    int cs = -1;  // first level of the fused coarse cycle
    long long off = 0, len = 0;
    double rel_tol = 0, f_inf = 0;
    Clock::time_point t_add;
    // level 0 (and level 1 for the coefficient setup) of this problem alone
    DevBuf<RBox> rb0, rb1;
    DevBuf<Tile> t0;
    int nt0 = 0;
    TileShape sh0{};
    DevBuf<GhostCopy> face0[2], full_even0;
    DevBuf<int> cbox0;
    DevBuf<Tile> tface[3];
    int ntface[3] = {0, 0, 0};
    TileShape shface[3]{};
    std::vector<std::unique_ptr<PFaces<double>>> f64;  // index = level (0 unused)
    std::vector<std::unique_ptr<PFaces<float>>> f32;
    size_t face_bytes = 0;
    std::vector<std::unique_ptr<CList>> clist;  // index = level - cs
    int res0 = 0;
    Grid grid0() const { return Grid{rb0.p, t0.p, nt0, sh0, L[0].push ? 1 : 0, nullptr, 0, res0}; }
    XGrid face_grid(int d) const {
        return XGrid{rb0.p, rb1.p, cbox0.p, tface[d].p, ntface[d], shface[d], 0, nullptr, 0};
    }
};

// Launch structures of one level index over the running problems.
struct BLevel {
    DevBuf<RBox> rb;
    DevBuf<Tile> tcol, tdown;
    int ntcol = 0, ntdown = 0;
    TileShape shcol{}, shdown{};
    DevBuf<int> cbox;
    bool push = true;
    DevBuf<GhostCopy> face[2], fullc;  // face ghosts of l; every ghost of l + 1
    long long nface[2] = {0, 0}, nfullc = 0;
    DevBuf<ZeroRange> zr;  // level l + 1 of the problems tiled at l
    int nzr = 0;
    long long zmax = 0;
    DevBuf<FaceArrays<double>> fat64;  // by slot
    DevBuf<FaceArrays<float>> fat32;
    int flip = 0;
    int res = 1;
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
    size_t budget = 0, arena_bytes = 0, face_budget = 0, face_used = 0;
    long long cap = 0;  // arena elements
    Ranges ranges;
    DevBuf<double> u64, f64, b64;
    DevBuf<float> u32, f32, b32;
    // per slot
    DevBuf<int> active, nactive;
    DevBuf<BatchSlot> st;
    DevBuf<double> norms, hist, hist_l2;
    int* h_active = nullptr;
    int* h_nactive = nullptr;
    BatchSlot* h_st = nullptr;
    std::vector<std::unique_ptr<Problem>> slots;
    std::deque<int> free_slots;
    int64_t next_id = 1;
    std::deque<Done> done;
    // launch structures of the running set
    bool dirty = true;
    std::vector<int> members;
    DevBuf<int> d_members;
    std::vector<BLevel> lev;
    int lmax = 0;
    DevBuf<int> tstart, segslot;
    int nseg = 0;
    DevBuf<double> partials, scratch;
    DevBuf<ZeroRange> z0;
    int nz0 = 0;
    long long z0max = 0;
    DevBuf<CoarseCycle<double>> cc64;
    DevBuf<CoarseCycle<float>> cc32;
    std::vector<CoarseCycle<double>> cc64_host;
    std::vector<CoarseCycle<float>> cc32_host;
    int ncc = 0;
    bool use_graph = true;
    bool inflight = false;  // cycles launched and not yet collected
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // the batch's own stream (default priority): graphs cannot be captured on
    // the legacy default stream a context may use
    hipStream_t stream = nullptr;
    ~bxmg_batch_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (stream) (void)hipStreamDestroy(stream);
        if (h_active) (void)hipHostFree(h_active);
        if (h_nactive) (void)hipHostFree(h_nactive);
        if (h_st) (void)hipHostFree(h_st);
    }
};

namespace {

// ------------------------------------------------------- problem layout
// The problem's hierarchy, its coarse-cycle start, and its element count;
// false if it cannot run in a batch.
bool plan_problem(const bxmg_ba_s* ba, double h0, Problem& p, long long* len, std::string* why) {
    p.dom = ba->dom;
    for (int d = 0; d < 3; ++d) p.per[d] = ba->per[d];
    const std::vector<LevelBoxes> lb = make_hierarchy(ba->dom, ba->boxes);
    if (!bottom_fits(lb.back().dom)) {
        if (why) *why = "bottom level above 4096 cells";
        return false;
    }
    const size_t nl = lb.size();
    p.cs = -1;
    for (size_t l = 1; l < nl; ++l) {
        bool ok = nl - l <= (size_t)kMaxCoarseLevels;
        for (size_t m = l; m < nl && ok; ++m) ok = lb[m].boxes.size() == 1 && lb[m].dom.cells() <= kMaxBottomCells;
        if (ok) { p.cs = (int)l; break; }
    }
    if (p.cs < 0) {
        if (why) *why = "the trailing levels are not single boxes of at most 4096 cells";
        return false;
    }
    p.L.clear();
    long long off = 0;
    double h = h0;
    for (size_t l = 0; l < nl; ++l) {
        PLevel v;
        v.dom = lb[l].dom;
        v.h = h;
        h *= 2.0;
        v.boxes = lb[l].boxes;
        v.rb = rb_layout(v.boxes, 1, v.h, &v.nelem);
        v.push = face_neighbours(v.dom, p.per, v.boxes, v.rb);
        v.off = off;
        off += v.nelem;
        if (l + 1 < nl) v.cbox = coarse_owner(v.boxes, lb[l + 1].boxes);
        p.L.push_back(std::move(v));
    }
    *len = (off + 63) / 64 * 64;
    return true;
}

size_t face_bytes_of(const Problem& p, int es) {
    size_t n = 0;
    for (size_t l = 1; l < p.L.size(); ++l) {
        const Box& D = p.L[l].dom;
        for (int d = 0; d < 3; ++d) n += (size_t)(D.n(0) + (d == 0)) * (D.n(1) + (d == 1)) * (D.n(2) + (d == 2));
    }
    return n * es;
}

// Places the problem at arena offset `base`: absolute box bases, ghost lists.
void place_problem(Problem& p, long long base, bool var) {
    p.off = base;
    for (size_t l = 0; l < p.L.size(); ++l) {
        PLevel& v = p.L[l];
        v.off += base;
        for (auto& r : v.rb) r.base += v.off;
        const std::vector<Tag> faces = build_tags(v.dom, p.per, v.boxes, 1, true, 2, true);
        v.face[0] = ghost_list(faces, v.rb, 1);
        v.face[1] = ghost_list(faces, v.rb, 2);
        v.full = ghost_list(build_tags(v.dom, p.per, v.boxes, 1, false, 2, true), v.rb, 3);
    }
    // coarse-cycle levels: lists relative to the level start
    p.clist.clear();
    for (size_t l = (size_t)p.cs; l < p.L.size(); ++l) {
        PLevel& v = p.L[l];
        auto rel = [&](const std::vector<GhostCopy>& a) {
            std::vector<GhostCopy> o(a);
            for (auto& g : o) {
                g.dst -= (uint32_t)v.off;
                g.src = ((g.src & 0x7fffffffu) - (uint32_t)v.off) | (g.src & 0x80000000u);
            }
            return o;
        };
        auto c = std::make_unique<CList>();
        c->face[0].upload(rel(v.face[0]));
        c->face[1].upload(rel(v.face[1]));
        c->full.upload(rel(v.full));
        p.clist.push_back(std::move(c));
    }
    // level 0 alone: setup, norms of f, final conversion
    p.rb0.upload(p.L[0].rb);
    p.rb1.upload(p.L[1].rb);
    p.face0[0].upload(p.L[0].face[0]);
    p.face0[1].upload(p.L[0].face[1]);
    p.cbox0.upload(p.L[0].cbox);
    if (var) {
        std::vector<RBox> rb = p.L[0].rb;
        p.full_even0.upload(ghost_list(build_tags(p.L[0].dom, p.per, p.L[0].boxes, 1, false, 2, false), rb, 3));
    }
}

void problem_tiles(Problem& p, int zc, int zc_planes, int res, bool var) {
    p.res0 = (res && boxes_fit_res(p.L[0].rb)) ? 1 : 0;
    TileSet ts = make_tiles(colour_extents(p.L[0].boxes), zc);
    if (ts.sh.lz == 0) ts = make_tiles(colour_extents(p.L[0].boxes), zc_planes);
    p.t0.upload(ts.tiles);
    p.nt0 = (int)ts.tiles.size();
    p.sh0 = ts.sh;
    if (var)
        for (int d = 0; d < 3; ++d) {
            TileSet tf = make_tiles(coarse_extents(p.L[0].boxes, p.L[0].dom, d), zc);
            p.tface[d].upload(tf.tiles);
            p.ntface[d] = (int)tf.tiles.size();
            p.shface[d] = tf.sh;
        }
}

template <class T>
void alloc_faces(Problem& p, std::vector<std::unique_ptr<PFaces<T>>>& F) {
    F.clear();
    F.resize(p.L.size());
    for (size_t l = 1; l < p.L.size(); ++l) {
        F[l] = std::make_unique<PFaces<T>>();
        const Box& D = p.L[l].dom;
        for (int d = 0; d < 3; ++d) {
            F[l]->c[d].alloc((size_t)(D.n(0) + (d == 0)) * (D.n(1) + (d == 1)) * (D.n(2) + (d == 2)));
            F[l]->view.c[d] = F[l]->c[d].p;
            F[l]->view.dlo[d] = D.lo[d];
            F[l]->view.n[d] = D.n(d);
        }
    }
}

// face arrays of levels >= 1 from the level-0 cell beta (as the single-problem setup)
template <class T>
void setup_faces(hipStream_t s, Problem& p, std::vector<std::unique_ptr<PFaces<T>>>& F, T* beta_arena) {
    HIPCHK(launch_fill_rb(s, beta_arena, sizeof(T) == 4, p.full_even0.p, (long long)p.full_even0.n));
    for (size_t l = 1; l < p.L.size(); ++l)
        for (int d = 0; d < 3; ++d) {
            T* dst = F[l]->c[d].p;
            if (l == 1) HIPCHK(launch_faces_from_cells<T>(s, p.face_grid(d), beta_arena, d, F[l]->view, dst));
            else HIPCHK(launch_faces_coarsen<T>(s, F[l - 1]->view, F[l]->view, d, dst));
        }
}

template <class T>
CoarseCycle<T> coarse_desc(const bxmg_batch_s* b, const Problem& p, T* u, T* f,
                           const std::vector<std::unique_ptr<PFaces<T>>>* F) {
    CoarseCycle<T> cc;
    std::memset(&cc, 0, sizeof cc);
    cc.nlev = (int)p.L.size() - p.cs;
    cc.nu1 = b->P.nu1;
    cc.nu2 = b->P.nu2;
    cc.prolong = b->P.prolong;
    for (int d = 0; d < 3; ++d) cc.per[d] = p.per[d];
    cc.pid = p.slot;
    cc.rtol = b->P.bottom_rtol;
    cc.iters = nullptr;
    for (int m = 0; m < cc.nlev; ++m) {
        const PLevel& v = p.L[p.cs + m];
        CoarseLevel<T>& c = cc.L[m];
        c.box = v.rb[0];
        c.box.base -= v.off;
        c.u = u + v.off;
        c.f = f + v.off;
        const CList& cl = *p.clist[m];
        for (int q = 0; q < 2; ++q) { c.face[q] = cl.face[q].p; c.nface[q] = (long long)cl.face[q].n; }
        c.full = cl.full.p;
        c.nfull = (long long)cl.full.n;
        c.nelem = v.nelem;
        c.h = v.h;
        if (F && p.cs + m >= 1) {
            c.fa = (*F)[p.cs + m]->view;
        } else {
            for (int d = 0; d < 3; ++d) { c.fa.c[d] = nullptr; c.fa.dlo[d] = 0; c.fa.n[d] = 0; }
        }
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
    b->d_members.upload(b->members);
    b->lev.clear();
    b->lmax = 0;
    b->ncc = 0;
    b->nseg = 0;
    b->dirty = false;
    if (b->members.empty()) return;
    size_t depth = 0;
    for (int s : b->members) {
        depth = std::max(depth, b->slots[s]->L.size());
        b->lmax = std::max(b->lmax, b->slots[s]->cs);
    }
    b->lev.resize(depth);
    std::vector<std::vector<int>> first(depth, std::vector<int>(b->max_slots, -1));  // first box of slot at level
    std::vector<std::vector<RBox>> rbs(depth);
    for (size_t l = 0; l < depth; ++l)
        for (int s : b->members) {
            const Problem& p = *b->slots[s];
            if (l >= p.L.size()) continue;
            first[l][s] = (int)rbs[l].size();
            for (const RBox& r0 : p.L[l].rb) {
                RBox r = r0;
                r.pid = s;
                for (int q = 0; q < 6; ++q)
                    if (r.nb[q] >= 0) r.nb[q] += first[l][s];
                rbs[l].push_back(r);
            }
        }
    const int zc = b->ctx->zc, zcp = b->ctx->zc_planes;
    std::vector<int> tstart{0}, segslot;
    for (size_t l = 0; l < depth; ++l) {
        BLevel& B = b->lev[l];
        B.rb.upload(rbs[l]);
        B.res = (b->ctx->res && boxes_fit_res(rbs[l])) ? 1 : 0;
        if ((int)l >= b->lmax) continue;
        // tiled problems at l: colour tiles, transfer tiles, lists
        std::vector<std::array<int, 3>> ecol, edown;
        std::vector<int> gcol, gdown, cbox;
        std::vector<GhostCopy> face[2], fullc;
        std::vector<ZeroRange> zr;
        B.push = true;
        for (int s : b->members) {
            const Problem& p = *b->slots[s];
            if ((int)l >= p.cs) continue;
            const PLevel& v = p.L[l];
            const auto ce = colour_extents(v.boxes);
            const auto de = coarse_extents(v.boxes, v.dom, -1);
            for (size_t q = 0; q < v.boxes.size(); ++q) {
                ecol.push_back(ce[q]);
                gcol.push_back(first[l][s] + (int)q);
                edown.push_back(de[q]);
                gdown.push_back(first[l][s] + (int)q);
                cbox.push_back(first[l + 1][s] + v.cbox[q]);
            }
            B.push = B.push && v.push;
            for (int c = 0; c < 2; ++c) face[c].insert(face[c].end(), v.face[c].begin(), v.face[c].end());
            const PLevel& w = p.L[l + 1];
            fullc.insert(fullc.end(), w.full.begin(), w.full.end());
            zr.push_back(ZeroRange{w.off, w.nelem, s, 0});
            B.zmax = std::max(B.zmax, w.nelem);
        }
        TileSet tc = make_tiles(ecol, zc);
        if (tc.sh.lz == 0) tc = make_tiles(ecol, zcp);
        for (auto& t : tc.tiles) t.box = gcol[t.box];
        TileSet td = make_tiles(edown, zc);
        std::vector<int> cb(td.tiles.size());
        // the transfer kernels index cbox by the fine box of the tile
        std::vector<int> cbox_full(rbs[l].size(), -1);
        for (size_t q = 0; q < gdown.size(); ++q) cbox_full[gdown[q]] = cbox[q];
        for (auto& t : td.tiles) t.box = gdown[t.box];
        B.tcol.upload(tc.tiles);
        B.ntcol = (int)tc.tiles.size();
        B.shcol = tc.sh;
        B.tdown.upload(td.tiles);
        B.ntdown = (int)td.tiles.size();
        B.shdown = td.sh;
        B.cbox.upload(cbox_full);
        if (!B.push)
            for (int c = 0; c < 2; ++c) { B.face[c].upload(face[c]); B.nface[c] = (long long)face[c].size(); }
        B.fullc.upload(fullc);
        B.nfullc = (long long)fullc.size();
        B.zr.upload(zr);
        B.nzr = (int)zr.size();
        if (l == 0) {
            // per-problem segments of the level-0 tiles (tiles run problem-major)
            int cur = -1;
            for (size_t t = 0; t < tc.tiles.size(); ++t) {
                const int s = rbs[0][tc.tiles[t].box].pid;
                if (s != cur) {
                    if (cur >= 0) tstart.push_back((int)t);
                    segslot.push_back(s);
                    cur = s;
                }
            }
            tstart.push_back((int)tc.tiles.size());
        }
    }
    b->tstart.upload(tstart);
    b->segslot.upload(segslot);
    b->nseg = (int)segslot.size();
    b->partials.alloc(3 * (size_t)std::max(1, b->lev[0].ntcol) + 8);
    // level-0 ranges (the FP32 correction starts from zero every cycle)
    std::vector<ZeroRange> z0;
    b->z0max = 0;
    for (int s : b->members) {
        const PLevel& v = b->slots[s]->L[0];
        z0.push_back(ZeroRange{v.off, v.nelem, s, 0});
        b->z0max = std::max(b->z0max, v.nelem);
    }
    b->z0.upload(z0);
    b->nz0 = (int)z0.size();
    // coefficient tables by slot
    if (b->var)
        for (size_t l = 1; l < depth; ++l) {
            BLevel& B = b->lev[l];
            if (b->prec == 0) {
                std::vector<FaceArrays<double>> t(b->max_slots);
                std::memset(t.data(), 0, t.size() * sizeof(t[0]));
                for (int s : b->members)
                    if (l < b->slots[s]->L.size()) t[s] = b->slots[s]->f64[l]->view;
                B.fat64.upload(t);
            } else {
                std::vector<FaceArrays<float>> t(b->max_slots);
                std::memset(t.data(), 0, t.size() * sizeof(t[0]));
                for (int s : b->members)
                    if (l < b->slots[s]->L.size()) t[s] = b->slots[s]->f32[l]->view;
                B.fat32.upload(t);
            }
        }
    // fused coarse cycles
    b->cc64_host.clear();
    b->cc32_host.clear();
    for (int s : b->members) {
        const Problem& p = *b->slots[s];
        if (b->prec == 0) b->cc64_host.push_back(coarse_desc<double>(b, p, b->u64.p, b->f64.p, b->var ? &p.f64 : nullptr));
        else b->cc32_host.push_back(coarse_desc<float>(b, p, b->u32.p, b->f32.p, b->var ? &p.f32 : nullptr));
    }
    if (b->prec == 0) b->cc64.upload(b->cc64_host);
    else b->cc32.upload(b->cc32_host);
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
    return (b->var && l >= 1) ? b->lev[l].fat64.p : nullptr;
}
template <>
const FaceArrays<float>* level_fat<float>(bxmg_batch_s* b, size_t l) {
    return (b->var && l >= 1) ? b->lev[l].fat32.p : nullptr;
}
template <class T>
const CoarseCycle<T>* coarse_descs(bxmg_batch_s* b);
template <>
const CoarseCycle<double>* coarse_descs<double>(bxmg_batch_s* b) { return b->cc64.p; }
template <>
const CoarseCycle<float>* coarse_descs<float>(bxmg_batch_s* b) { return b->cc32.p; }

Grid level_grid(bxmg_batch_s* b, size_t l) {
    BLevel& B = b->lev[l];
    Grid g{B.rb.p, B.tcol.p, B.ntcol, B.shcol, B.push ? 1 : 0, b->active.p, B.flip, B.res};
    B.flip ^= 1;
    return g;
}

XGrid level_xgrid(bxmg_batch_s* b, size_t l) {
    BLevel& B = b->lev[l];
    XGrid x{B.rb.p, b->lev[l + 1].rb.p, B.cbox.p, B.tdown.p, B.ntdown, B.shdown, B.push ? 1 : 0, b->active.p, B.flip};
    B.flip ^= 1;
    return x;
}

template <class T>
void b_smooth(bxmg_batch_s* b, hipStream_t s, size_t l, int nsweeps) {
    BLevel& B = b->lev[l];
    T* u = arena_u<T>(b);
    for (int k = 0; k < nsweeps; ++k)
        for (int c = 0; c < 2; ++c) {
            if (!B.push) HIPCHK(launch_fill_rb(s, u, sizeof(T) == 4, B.face[c ^ 1].p, B.nface[c ^ 1]));
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
            HIPCHK(launch_fill_rb(s, u, f32, B.face[0].p, B.nface[0]));
            HIPCHK(launch_fill_rb(s, u, f32, B.face[1].p, B.nface[1]));
        }
        HIPCHK(launch_resid_restrict<T>(s, level_xgrid(b, l), u, f, arena_beta<T>(b, l), level_fat<T>(b, l), f));
        HIPCHK(launch_zero_ranges<T>(s, u, B.zr.p, B.nzr, B.zmax, b->active.p));
    }
    HIPCHK(launch_coarse_cycle<T>(s, coarse_descs<T>(b), b->ncc, b->active.p, b->var));
    for (int l = b->lmax - 1; l >= 0; --l) {
        BLevel& B = b->lev[l];
        HIPCHK(launch_fill_rb(s, u, f32, B.fullc.p, B.nfullc));
        HIPCHK(launch_prolong<T>(s, level_grid(b, l), b->lev[l + 1].rb.p, B.cbox.p, u, u, b->P.prolong));
        b_smooth<T>(b, s, l, b->P.nu2);
    }
}

// One batch cycle: FP64 residual and per-problem norms, the stop test, and
// the V-cycle (FP64, or FP32 correction added to the FP64 solution).
void enqueue_cycle(bxmg_batch_s* b, hipStream_t s) {
    const double* beta0 = b->var ? b->b64.p : nullptr;
    if (b->prec == 0)
        HIPCHK(launch_resid<double, double>(s, level_grid(b, 0), b->u64.p, b->f64.p, beta0, nullptr, (double*)nullptr,
                                            b->partials.p));
    else
        HIPCHK(launch_resid<double, float>(s, level_grid(b, 0), b->u64.p, b->f64.p, beta0, nullptr, b->f32.p,
                                           b->partials.p));
    HIPCHK(launch_norm_seg(s, b->partials.p, b->tstart.p, b->segslot.p, b->nseg, b->active.p, b->norms.p));
    HIPCHK(launch_batch_check(s, b->d_members.p, (int)b->members.size(), b->norms.p, b->st.p, b->active.p,
                              b->hist.p, b->hist_l2.p, b->nactive.p));
    if (b->prec == 0) {
        b_vcycle<double>(b, s);
    } else {
        HIPCHK(launch_zero_ranges<float>(s, b->u32.p, b->z0.p, b->nz0, b->z0max, b->active.p));
        b_vcycle<float>(b, s);
        HIPCHK(launch_add_f32(s, level_grid(b, 0), b->u64.p, b->u32.p));
    }
}

// -------------------------------------------------------- finish / release
void release_problem(bxmg_batch_s* b, int s) {
    Problem& p = *b->slots[s];
    if (p.len > 0) b->ranges.give(p.off, p.len);
    b->face_used -= p.face_bytes;
    b->slots[s].reset();
    b->free_slots.push_back(s);
}

// Writes the solution of a stopped problem into its phi and queues its result.
void grow(DevBuf<double>& d, size_t n) {
    if (d.n < n) d.alloc(n);
}

// convert == false: phi is left as it was (non-finite right-hand side)
void finish_problem(bxmg_batch_s* b, int s, hipStream_t st, bool convert) {
    Problem& p = *b->slots[s];
    const BatchSlot S = b->h_st[s];
    Done d;
    d.id = p.id;
    std::memset(&d.info, 0, sizeof d.info);
    d.info.status = S.status;
    d.info.cycles = S.cycles;
    d.info.levels = (int)p.L.size();
    d.info.nhist = std::min(S.nhist, kHist);
    d.info.f_inf = p.f_inf;
    if (d.info.nhist > 0) {
        HIPCHK(hipMemcpy(d.info.hist, b->hist.p + (size_t)s * kHist, d.info.nhist * sizeof(double),
                         hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(d.info.hist_l2, b->hist_l2.p + (size_t)s * kHist, d.info.nhist * sizeof(double),
                         hipMemcpyDeviceToHost));
        d.info.rel_resid_inf = d.info.hist[d.info.nhist - 1];
        d.info.resid_l2 = d.info.hist_l2[d.info.nhist - 1];
    }
    if (convert) {
        const Grid g0 = p.grid0();
        if (p.per[0] && p.per[1] && p.per[2]) {
            grow(b->scratch, 3 * (size_t)p.nt0 + 8);
            HIPCHK(launch_mean_sub(st, g0, b->u64.p, b->scratch.p));
        }
        HIPCHK(launch_rb_to_fab(st, g0, b->u64.p, (double*)p.phi->data, p.phi->d_fboxes.p));
        HIPCHK(hipStreamSynchronize(st));
    }
    d.info.seconds = std::chrono::duration<double>(Clock::now() - p.t_add).count();
    b->done.push_back(d);
    release_problem(b, s);
}

size_t arena_bytes_per_elem(int prec, bool var) {
    size_t e = 16;              // u, f FP64
    if (prec == 1) e += 8;      // u, f FP32
    if (var) e += prec ? 12 : 8;  // beta FP64 (+ FP32)
    return e;
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
    b->var = var != 0;
    b->prec = b->P.precision;
    b->max_slots = max_problems;
    b->budget = hbm_budget_bytes;
    // coefficient faces of levels >= 1 take about 3/7 of a level-0 array
    const size_t per = arena_bytes_per_elem(b->prec, b->var);
    const size_t fes = b->var ? (b->prec ? 4 : 8) : 0;
    const double face_share = b->var ? (double)fes * 0.45 / (double)(per + fes * 0.45) : 0.0;
    b->face_budget = (size_t)(face_share * (double)hbm_budget_bytes);
    long long cap = (long long)((hbm_budget_bytes - b->face_budget) / per);
    cap = std::min<long long>(cap, 0x7fffffffLL) / 64 * 64;
    if (cap < 64) return fail(BXMG_EINVAL, "batch_create: budget too small");
    b->cap = cap;
    b->arena_bytes = (size_t)cap * per;
    std::lock_guard<std::mutex> lock(ctx->mu);
    try {
        HIPCHK(hipSetDevice(ctx->device));
        HIPCHK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        b->u64.alloc(cap);
        b->f64.alloc(cap);
        if (b->prec == 1) { b->u32.alloc(cap); b->f32.alloc(cap); }
        if (b->var) { b->b64.alloc(cap); if (b->prec == 1) b->b32.alloc(cap); }
        b->active.alloc(max_problems);
        HIPCHK(hipMemset(b->active.p, 0, max_problems * sizeof(int)));
        b->nactive.alloc(1);
        b->st.alloc(max_problems);
        b->norms.alloc(3 * (size_t)max_problems);
        b->hist.alloc((size_t)max_problems * kHist);
        b->hist_l2.alloc((size_t)max_problems * kHist);
        HIPCHK(hipHostMalloc((void**)&b->h_active, max_problems * sizeof(int)));
        HIPCHK(hipHostMalloc((void**)&b->h_nactive, sizeof(int)));
        HIPCHK(hipHostMalloc((void**)&b->h_st, max_problems * sizeof(BatchSlot)));
        std::memset(b->h_active, 0, max_problems * sizeof(int));
    } catch (HipError& e) {
        return fail(e.e == hipErrorOutOfMemory ? BXMG_ENOMEM : BXMG_EDEVICE,
                    std::string("batch_create: ") + hipGetErrorString(e.e));
    }
    b->ranges.init(cap);
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
    Problem p;
    long long len = 0;
    try {
        if (!plan_problem(ba, 1.0, p, &len, nullptr)) return 0;
    } catch (std::exception&) {
        return 0;
    }
    return (size_t)len * arena_bytes_per_elem(b->prec, b->var) + (b->var ? face_bytes_of(p, b->prec ? 4 : 8) : 0);
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
    auto p = std::make_unique<Problem>();
    const double h = (b->P.dx > 0) ? b->P.dx : 1.0 / ba->dom.n(0);
    long long len = 0;
    std::string why;
    try {
        if (!plan_problem(ba, h, *p, &len, &why)) return fail(BXMG_EINVAL, "batch_add: " + why);
    } catch (std::exception& e) {
        return fail(BXMG_EINVAL, std::string("batch_add: ") + e.what());
    }
    const size_t fbytes = b->var ? face_bytes_of(*p, b->prec ? 4 : 8) : 0;
    if (b->free_slots.empty()) return fail(BXMG_EBUSY, "batch_add: every slot is taken");
    if (b->face_used + fbytes > b->face_budget) return fail(BXMG_EBUSY, "batch_add: coefficient storage is full");
    if (len > b->cap) return fail(BXMG_EINVAL, "batch_add: the problem is larger than the whole arena");
    const long long base = b->ranges.take(len);
    if (base < 0) return fail(BXMG_EBUSY, "batch_add: the arena has no free range of this size");
    const int slot = b->free_slots.front();
    p->slot = slot;
    p->len = len;
    p->id = b->next_id;
    p->phi = phi;
    p->rhs = rhs;
    p->beta = beta;
    p->rel_tol = rel_tol > 0 ? rel_tol : b->P.rel_tol;
    p->t_add = Clock::now();
    hipStream_t s = b->stream;
    try {
        HIPCHK(hipSetDevice(b->ctx->device));
        HIPCHK(hipStreamSynchronize(b->ctx->stream));  // the caller's writes to phi, rhs, beta
        place_problem(*p, base, b->var);
        problem_tiles(*p, b->ctx->zc, b->ctx->zc_planes, b->ctx->res, b->var);
        const Grid g0 = p->grid0();
        const PLevel& L0 = p->L[0];
        HIPCHK(launch_fab_to_rb(s, g0, (const double*)phi->data, phi->d_fboxes.p, b->u64.p, false));
        HIPCHK(launch_fab_to_rb(s, g0, (const double*)rhs->data, rhs->d_fboxes.p, b->f64.p, false));
        if (b->var) {
            HIPCHK(launch_fab_to_rb(s, g0, (const double*)beta->data, beta->d_fboxes.p, b->b64.p, false));
            p->face_bytes = fbytes;
            if (b->prec == 0) {
                alloc_faces<double>(*p, p->f64);
                setup_faces<double>(s, *p, p->f64, b->b64.p);
            } else {
                alloc_faces<float>(*p, p->f32);
                HIPCHK(launch_fill_rb(s, b->b64.p, false, p->full_even0.p, (long long)p->full_even0.n));
                HIPCHK(launch_cast_f32(s, b->b64.p + L0.off, b->b32.p + L0.off, L0.nelem));
                setup_faces<float>(s, *p, p->f32, b->b32.p);
            }
        }
        // ghosts of the converted guess (later producers keep them current)
        HIPCHK(launch_fill_rb(s, b->u64.p, false, p->face0[0].p, (long long)p->face0[0].n));
        HIPCHK(launch_fill_rb(s, b->u64.p, false, p->face0[1].p, (long long)p->face0[1].n));
        grow(b->scratch, 3 * (size_t)p->nt0 + 8);
        HIPCHK(launch_field_norm(s, g0, b->f64.p, b->scratch.p));
        HIPCHK(launch_norm_final(s, b->scratch.p, p->nt0, b->scratch.p + 3 * (size_t)p->nt0));
        double fn[3];
        HIPCHK(hipMemcpyAsync(fn, b->scratch.p + 3 * (size_t)p->nt0, sizeof fn, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        BatchSlot S{};
        S.fnorm = fn[0];
        S.rel_tol = p->rel_tol;
        S.abs_tol = b->P.abs_tol;
        S.max_cycles = b->P.max_cycles;
        S.fixed_cycles = b->P.fixed_cycles;
        p->f_inf = fn[2] > 0 ? NAN : fn[0];
        int act = 1;
        if (fn[2] > 0) { S.status = BXMG_ENONFINITE; act = 0; }
        else if (!(fn[0] > 0.0)) act = 0;  // f == 0: u stays the guess
        HIPCHK(hipMemcpy(b->st.p + slot, &S, sizeof S, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(b->active.p + slot, &act, sizeof act, hipMemcpyHostToDevice));
        b->free_slots.pop_front();
        b->face_used += p->face_bytes;
        b->slots[slot] = std::move(p);
        b->h_active[slot] = act;
        b->h_st[slot] = S;
        ++b->next_id;
        *id = b->slots[slot]->id;
        if (act) b->dirty = true;
        else finish_problem(b, slot, s, fn[2] == 0);
    } catch (HipError& e) {
        if (!b->slots[slot]) b->ranges.give(base, len);
        return fail(e.e == hipErrorOutOfMemory ? BXMG_ENOMEM : BXMG_EDEVICE,
                    std::string("batch_add: ") + e.where + ": " + hipGetErrorString(e.e));
    } catch (std::exception& e) {
        if (!b->slots[slot]) b->ranges.give(base, len);
        return fail(BXMG_EINVAL, std::string("batch_add: ") + e.what());
    }
    return BXMG_OK;
}

static bxmg_status batch_launch(bxmg_batch b, int32_t ncycles) {
    if (ncycles < 1) return fail(BXMG_EINVAL, "batch_launch: ncycles < 1");
    if (b->inflight) return fail(BXMG_EBUSY, "batch_launch: the cycles launched before are not collected");
    hipStream_t s = b->stream;
    try {
        HIPCHK(hipSetDevice(b->ctx->device));
        if (b->dirty) rebuild(b);
        if (b->members.empty()) return BXMG_OK;
        if (b->use_graph && !b->exec) {
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
            for (int m : b->members)
                if (b->slots[m] && !b->h_active[m]) {
                    finish_problem(b, m, s, true);
                    b->dirty = true;
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
            try {
                HIPCHK(hipSetDevice(b->ctx->device));
                HIPCHK(hipStreamSynchronize(b->stream));
                const int zero = 0;
                HIPCHK(hipMemcpy(b->active.p + s, &zero, sizeof zero, hipMemcpyHostToDevice));
            } catch (HipError& e) {
                return fail(BXMG_EDEVICE, std::string("batch_remove: ") + hipGetErrorString(e.e));
            }
            b->h_active[s] = 0;
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
    long long free_el = 0;
    for (auto& r : b->ranges.free) free_el += r.second;
    if (bytes_used) *bytes_used = (size_t)(b->cap - free_el) * per + b->face_used;
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
