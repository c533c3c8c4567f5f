// Host side of libbxmg: BoxArrays, MultiFabs, cached ghost-copy plans, the
// multigrid hierarchy and the V-cycle driver, behind the C ABI of bxmg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bxmg.h"
#include "bxmg_internal.h"

using namespace bxmg;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static bxmg_status fail(bxmg_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

struct HipError {
    hipError_t e;
    const char* where;
};

#define HIPCHK(x)                                          \
    do {                                                   \
        hipError_t e_ = (x);                               \
        if (e_ != hipSuccess) throw HipError{e_, #x};      \
    } while (0)

// -------------------------------------------------------------- box algebra
namespace {

struct Box {
    int lo[3], hi[3];
    int n(int d) const { return hi[d] - lo[d] + 1; }
    long long cells() const { return (long long)n(0) * n(1) * n(2); }
    bool ok() const { return lo[0] <= hi[0] && lo[1] <= hi[1] && lo[2] <= hi[2]; }
    bool contains(const Box& b) const {
        for (int d = 0; d < 3; ++d)
            if (b.lo[d] < lo[d] || b.hi[d] > hi[d]) return false;
        return true;
    }
};

Box intersect(const Box& a, const Box& b) {
    Box c;
    for (int d = 0; d < 3; ++d) { c.lo[d] = std::max(a.lo[d], b.lo[d]); c.hi[d] = std::min(a.hi[d], b.hi[d]); }
    return c;
}

int floor2(int a) { return a >> 1; }  // arithmetic shift: floor(a/2)

Box coarsen(const Box& b) {
    Box c;
    for (int d = 0; d < 3; ++d) { c.lo[d] = floor2(b.lo[d]); c.hi[d] = floor2(b.hi[d]); }
    return c;
}

std::vector<std::pair<int, int>> chop1(int lo, int n, int max_box) {
    int bf = 1;
    while (n % (bf * 2) == 0 && bf * 2 <= max_box) bf *= 2;
    const int piece = (max_box / bf) * bf;
    std::vector<std::pair<int, int>> out;
    for (int s = 0; s < n; s += piece) out.push_back({lo + s, lo + std::min(s + piece, n) - 1});
    return out;
}

bool domain_coarsenable(const Box& dom) {
    for (int d = 0; d < 3; ++d)
        if (dom.n(d) % 2 || dom.n(d) < 4 || (dom.lo[d] & 1)) return false;
    return true;
}

bool boxes_coarsenable(const std::vector<Box>& bs) {
    for (auto& b : bs)
        for (int d = 0; d < 3; ++d)
            if (b.n(d) % 2 || b.n(d) < 4 || (b.lo[d] & 1)) return false;
    return true;
}

struct LevelBoxes {
    Box dom;
    std::vector<Box> boxes;
};

std::vector<LevelBoxes> make_hierarchy(const Box& dom, const std::vector<Box>& b0) {
    std::vector<LevelBoxes> L{LevelBoxes{dom, b0}};
    while (domain_coarsenable(L.back().dom)) {
        LevelBoxes c;
        c.dom = coarsen(L.back().dom);
        if (boxes_coarsenable(L.back().boxes))
            for (auto& b : L.back().boxes) c.boxes.push_back(coarsen(b));
        else
            c.boxes.push_back(c.dom);
        L.push_back(c);
    }
    return L;
}

// --------------------------------------------------------- ghost-copy plans
// Region tags for the ghost cells of every box grown by ng.
// mode 0: FillBoundary (periodic shifts; ghosts outside a non-periodic face
//         are skipped);  mode 1: physical ghosts only (reflection into the
//         box's own grown data);  mode 2: FillBoundary and physical ghosts in
//         one plan (reflection + shift, read straight from the owning box).
// odd: sign -1 per reflected direction (homogeneous Dirichlet) or +1.
std::vector<Tag> build_tags(const Box& dom, const int per[3], const std::vector<Box>& boxes, int ng, bool cross,
                            int mode, bool odd) {
    std::vector<Tag> tags;
    long long prefix = 0;
    for (size_t b = 0; b < boxes.size(); ++b) {
        const Box& B = boxes[b];
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int dir[3] = {dx, dy, dz};
                    const int nnz = (dx != 0) + (dy != 0) + (dz != 0);
                    if (nnz == 0 || (cross && nnz != 1)) continue;
                    Box slab;
                    for (int d = 0; d < 3; ++d) {
                        if (dir[d] < 0) { slab.lo[d] = B.lo[d] - ng; slab.hi[d] = B.lo[d] - 1; }
                        else if (dir[d] > 0) { slab.lo[d] = B.hi[d] + 1; slab.hi[d] = B.hi[d] + ng; }
                        else { slab.lo[d] = B.lo[d]; slab.hi[d] = B.hi[d]; }
                    }
                    // split the slab per direction into below / inside / above the domain
                    std::vector<std::pair<int, int>> seg[3];
                    std::vector<int> kind[3];  // -1 below, 0 inside, +1 above
                    for (int d = 0; d < 3; ++d) {
                        const int a = slab.lo[d], z = slab.hi[d];
                        if (a < dom.lo[d]) { seg[d].push_back({a, std::min(z, dom.lo[d] - 1)}); kind[d].push_back(-1); }
                        if (std::max(a, dom.lo[d]) <= std::min(z, dom.hi[d])) {
                            seg[d].push_back({std::max(a, dom.lo[d]), std::min(z, dom.hi[d])});
                            kind[d].push_back(0);
                        }
                        if (z > dom.hi[d]) { seg[d].push_back({std::max(a, dom.hi[d] + 1), z}); kind[d].push_back(1); }
                    }
                    for (size_t s0 = 0; s0 < seg[0].size(); ++s0)
                        for (size_t s1 = 0; s1 < seg[1].size(); ++s1)
                            for (size_t s2 = 0; s2 < seg[2].size(); ++s2) {
                                const size_t si[3] = {s0, s1, s2};
                                Box piece;
                                int sgn[3], off[3], k[3];
                                int flips = 0, outside_nonper = 0;
                                bool skip = false;
                                for (int d = 0; d < 3; ++d) {
                                    piece.lo[d] = seg[d][si[d]].first;
                                    piece.hi[d] = seg[d][si[d]].second;
                                    k[d] = kind[d][si[d]];
                                    sgn[d] = 1;
                                    off[d] = 0;
                                    if (k[d] == 0) continue;
                                    if (per[d]) {
                                        if (mode == 1) continue;  // read own (already exchanged) ghost
                                        off[d] = (k[d] < 0) ? dom.n(d) : -dom.n(d);
                                    } else {
                                        ++outside_nonper;
                                        if (mode == 0) { skip = true; break; }
                                        sgn[d] = -1;
                                        off[d] = (k[d] < 0) ? 2 * dom.lo[d] - 1 : 2 * dom.hi[d] + 1;
                                        ++flips;
                                    }
                                }
                                if (skip) continue;
                                if (mode == 1 && outside_nonper == 0) continue;
                                // image of the piece
                                Box img;
                                for (int d = 0; d < 3; ++d) {
                                    const int a = sgn[d] * piece.lo[d] + off[d], z = sgn[d] * piece.hi[d] + off[d];
                                    img.lo[d] = std::min(a, z);
                                    img.hi[d] = std::max(a, z);
                                }
                                auto emit = [&](int sbox, const Box& I) {
                                    Tag t;
                                    t.dbox = (int)b;
                                    t.sbox = sbox;
                                    for (int d = 0; d < 3; ++d) {
                                        // preimage of I under s = sgn*x + off
                                        const int a = sgn[d] * (I.lo[d] - off[d]), z = sgn[d] * (I.hi[d] - off[d]);
                                        t.dlo[d] = std::min(a, z);
                                        t.n[d] = std::abs(z - a) + 1;
                                        t.sgn[d] = sgn[d];
                                        t.soff[d] = off[d];
                                    }
                                    t.neg = (odd && (flips & 1)) ? 1 : 0;
                                    t.pad = 0;
                                    t.prefix = prefix;
                                    prefix += (long long)t.n[0] * t.n[1] * t.n[2];
                                    tags.push_back(t);
                                };
                                if (mode == 1) {
                                    emit((int)b, img);  // mirror lies in the box's own grown region
                                } else {
                                    for (size_t q = 0; q < boxes.size(); ++q) {
                                        Box I = intersect(img, boxes[q]);
                                        if (I.ok()) emit((int)q, I);
                                    }
                                }
                            }
                }
    }
    return tags;
}

long long tag_cells(const std::vector<Tag>& t) {
    if (t.empty()) return 0;
    return t.back().prefix + (long long)t.back().n[0] * t.back().n[1] * t.back().n[2];
}

// Colour-cell work list: per box ceil(nx/2) x ny x nz threads.
std::vector<WorkBox> colour_work(const std::vector<Box>& boxes, long long* total) {
    std::vector<WorkBox> w;
    long long s = 0;
    for (size_t b = 0; b < boxes.size(); ++b) {
        WorkBox x;
        x.cstart = s;
        x.tn = (boxes[b].n(0) + 1) / 2;
        x.ny = boxes[b].n(1);
        x.nz = boxes[b].n(2);
        x.box = (int)b;
        x.cbox = -1;
        x.pad = 0;
        s += (long long)x.tn * x.ny * x.nz;
        w.push_back(x);
    }
    *total = s;
    return w;
}

// Coarse-cell work list of a fine level: per fine box its coarsened cells,
// with the index of the coarse box that contains them.  extra_d adds the
// high-boundary face layer in direction d for boxes touching dom.hi.
std::vector<WorkBox> coarse_work(const std::vector<Box>& fine, const std::vector<Box>& coarse, const Box& fdom,
                                 int extra_d, long long* total) {
    std::vector<WorkBox> w;
    long long s = 0;
    for (size_t b = 0; b < fine.size(); ++b) {
        const Box c = coarsen(fine[b]);
        int owner = -1;
        for (size_t q = 0; q < coarse.size(); ++q)
            if (coarse[q].contains(c)) { owner = (int)q; break; }
        WorkBox x;
        x.cstart = s;
        x.tn = c.n(0) + (extra_d == 0 && fine[b].hi[0] == fdom.hi[0]);
        x.ny = c.n(1) + (extra_d == 1 && fine[b].hi[1] == fdom.hi[1]);
        x.nz = c.n(2) + (extra_d == 2 && fine[b].hi[2] == fdom.hi[2]);
        x.box = (int)b;
        x.cbox = owner;
        x.pad = 0;
        s += (long long)x.tn * x.ny * x.nz;
        w.push_back(x);
    }
    *total = s;
    return w;
}

// RB layout of a level: per box two colour blocks, each 64-element aligned.
std::vector<RBox> rb_layout(const std::vector<Box>& boxes, int ng, long long* nelem) {
    std::vector<RBox> v;
    long long off = 0;
    for (auto& b : boxes) {
        RBox r;
        for (int d = 0; d < 3; ++d) {
            r.lo[d] = b.lo[d];
            r.hi[d] = b.hi[d];
            r.glo[d] = b.lo[d] - ng;
            r.G[d] = b.n(d) + 2 * ng;
        }
        r.H = (r.G[0] + 1) / 2;
        r.pid = 0;
        const long long half = (long long)r.H * r.G[1] * r.G[2];
        const long long padded = (half + 63) / 64 * 64;
        r.base = off;
        r.cstride = padded;
        off += 2 * padded;
        v.push_back(r);
    }
    *nelem = off;
    return v;
}

// ----------------------------------------------------------- device buffers
template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { if (p) (void)hipFree(p); }
    void alloc(size_t count) {
        if (p) { (void)hipFree(p); p = nullptr; }
        n = count;
        if (count) HIPCHK(hipMalloc((void**)&p, count * sizeof(T)));
    }
    void upload(const std::vector<T>& v) {
        alloc(v.size());
        if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    }
};

struct Plan {
    DevBuf<Tag> tags;
    int ntags = 0;
    long long cells = 0;
    void set(const std::vector<Tag>& t) {
        tags.upload(t);
        ntags = (int)t.size();
        cells = tag_cells(t);
    }
};

}  // namespace

// ============================================================ public handles
struct bxmg_ba_s {
    Box dom;
    int bc[3];
    int per[3];
    std::vector<Box> boxes;
    std::atomic<int> refs{1};
    uint64_t id;
};

static std::atomic<uint64_t> g_next_id{1};

static void ba_release(bxmg_ba_s* ba) {
    if (ba && --ba->refs == 0) delete ba;
}

struct Hier;

// Event pairs around the level-0 launches of one stage (bxmg_profile_stage).
struct Profiler {
    int stage = -1;
    std::vector<hipEvent_t> ev;
    size_t n = 0;
    long long launches = 0;
    double ms = 0.0;
    void mark(hipStream_t s) {
        if (n >= ev.size()) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            ev.push_back(e);
        }
        HIPCHK(hipEventRecord(ev[n++], s));
    }
    // after the stream has drained
    void harvest() {
        for (size_t i = 0; i + 1 < n; i += 2) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
            ms += t;
            ++launches;
        }
        n = 0;
    }
    ~Profiler() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

struct bxmg_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    Profiler prof;
    std::map<std::string, std::unique_ptr<Hier>> cache;
    double* h_norm = nullptr;  // pinned
    std::mutex mu;
};

struct bxmg_mf_s {
    bxmg_ctx ctx;
    bxmg_ba_s* ba;
    int ncomp, ng;
    bxmg_dtype dtype;
    void* data = nullptr;
    size_t bytes = 0;
    bool owned = false;
    std::vector<FBox> fboxes;
    DevBuf<FBox> d_fboxes;
    std::map<int, std::unique_ptr<Plan>> plans;  // key: mode*4 + cross*2 + odd
};

static size_t mf_layout(const bxmg_ba_s* ba, int ncomp, int ng, bxmg_dtype dt, std::vector<FBox>* out) {
    const size_t es = (dt == BXMG_F64) ? 8 : 4;
    const size_t align = 256 / es;
    size_t off = 0;
    for (auto& b : ba->boxes) {
        FBox f;
        long long n = 1;
        for (int d = 0; d < 3; ++d) {
            f.lo[d] = b.lo[d];
            f.hi[d] = b.hi[d];
            f.glo[d] = b.lo[d] - ng;
            f.G[d] = b.n(d) + 2 * ng;
            n *= f.G[d];
        }
        f.base = (long long)off;
        f.cs = n;
        if (out) out->push_back(f);
        off += (size_t)n * ncomp;
        off = (off + align - 1) / align * align;
    }
    return off * es;
}

static Plan* mf_plan(bxmg_mf_s* mf, int mode, bool cross, bool odd) {
    const int key = mode * 4 + (cross ? 2 : 0) + (odd ? 1 : 0);
    auto it = mf->plans.find(key);
    if (it != mf->plans.end()) return it->second.get();
    auto p = std::make_unique<Plan>();
    p->set(build_tags(mf->ba->dom, mf->ba->per, mf->ba->boxes, mf->ng, cross, mode, odd));
    Plan* raw = p.get();
    mf->plans[key] = std::move(p);
    return raw;
}

// ================================================================ hierarchy
namespace {

constexpr int kNormBlocks = 1024;

template <class T>
struct FaceSet {
    DevBuf<T> c[3];
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

struct Level {
    Box dom;
    double h;
    std::vector<Box> boxes;
    std::vector<RBox> rb;
    DevBuf<RBox> d_rb;
    long long nelem = 0;
    DevBuf<WorkBox> wcol;   // colour cells
    int nwcol = 0;
    long long ncol = 0;
    DevBuf<WorkBox> wdown;  // coarse cells of this level's boxes (to level+1)
    int nwdown = 0;
    long long ndown = 0;
    DevBuf<WorkBox> wface[3];  // coarse faces anchored in this level's boxes
    long long nface[3] = {0, 0, 0};
    Plan faces_odd;  // face ghosts, exchange + Dirichlet
    Plan full_odd;   // all ghosts, exchange + Dirichlet
    Plan full_even;  // all ghosts, exchange + even reflection (cell beta)
};

}  // namespace

struct Hier {
    int per[3];
    int precision;
    bool var;
    std::vector<std::unique_ptr<Level>> L;
    // FP64 storage: all levels (precision 0) or level 0 only (precision 1)
    std::vector<std::unique_ptr<DevBuf<double>>> u64, f64;
    std::vector<std::unique_ptr<DevBuf<float>>> u32, f32;
    DevBuf<double> beta64;
    DevBuf<float> beta32;
    std::vector<std::unique_ptr<FaceSet<double>>> faces64;  // index = level (0 unused)
    std::vector<std::unique_ptr<FaceSet<float>>> faces32;
    DevBuf<double> partials;  // 3*kNormBlocks + 3
    DevBuf<double> fnorm;     // 3
    DevBuf<int> iters;
    size_t bytes = 0;
};

static std::unique_ptr<Hier> build_hier(const bxmg_ba_s* ba, int precision, bool var, double h0) {
    auto H = std::make_unique<Hier>();
    for (int d = 0; d < 3; ++d) H->per[d] = ba->per[d];
    H->precision = precision;
    H->var = var;
    std::vector<LevelBoxes> lb = make_hierarchy(ba->dom, ba->boxes);
    double h = h0;
    for (size_t l = 0; l < lb.size(); ++l) {
        auto lv = std::make_unique<Level>();
        lv->dom = lb[l].dom;
        lv->h = h;
        h *= 2.0;
        lv->boxes = lb[l].boxes;
        lv->rb = rb_layout(lv->boxes, 1, &lv->nelem);
        lv->d_rb.upload(lv->rb);
        long long tot;
        auto wc = colour_work(lv->boxes, &tot);
        lv->wcol.upload(wc);
        lv->nwcol = (int)wc.size();
        lv->ncol = tot;
        if (l + 1 < lb.size()) {
            auto wd = coarse_work(lv->boxes, lb[l + 1].boxes, lv->dom, -1, &tot);
            lv->wdown.upload(wd);
            lv->nwdown = (int)wd.size();
            lv->ndown = tot;
            if (var)
                for (int d = 0; d < 3; ++d) {
                    auto wf = coarse_work(lv->boxes, lb[l + 1].boxes, lv->dom, d, &tot);
                    lv->wface[d].upload(wf);
                    lv->nface[d] = tot;
                }
        }
        lv->faces_odd.set(build_tags(lv->dom, H->per, lv->boxes, 1, true, 2, true));
        lv->full_odd.set(build_tags(lv->dom, H->per, lv->boxes, 1, false, 2, true));
        if (l == 0 && var) lv->full_even.set(build_tags(lv->dom, H->per, lv->boxes, 1, false, 2, false));
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
        }
    }
    H->partials.alloc(3 * kNormBlocks + 8);
    H->fnorm.alloc(4);
    H->iters.alloc(1);
    return H;
}

// ================================================================== driver
namespace {

struct Run {
    Hier* H;
    hipStream_t s;
    int nu1, nu2, prolong;
    double bottom_rtol;
    Profiler* prof = nullptr;
    // event brackets around level-0 launches of the profiled stage
    void pre(size_t l, int stage) { if (prof && prof->stage == stage && l == 0) prof->mark(s); }
    void post(size_t l, int stage) { if (prof && prof->stage == stage && l == 0) prof->mark(s); }
};

enum { kStageGS = 0, kStageResid = 1, kStageRestrict = 2, kStageProlong = 3, kStageFill = 4 };

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

template <class T>
void fill(Run& R, size_t l, T* data, const Plan& p, int cmask) {
    const Level& L = *R.H->L[l];
    R.pre(l, kStageFill);
    HIPCHK(launch_fill_rb(R.s, data, sizeof(T) == 4, L.d_rb.p, p.tags.p, p.ntags, p.cells, cmask));
    R.post(l, kStageFill);
}

template <class T>
void smooth(Run& R, size_t l, int nsweeps) {
    Hier* H = R.H;
    const Level& L = *H->L[l];
    T* u = lvl_u<T>(H, l);
    const T* f = lvl_f<T>(H, l);
    const T h2 = (T)(L.h * L.h);
    for (int s = 0; s < nsweeps; ++s)
        for (int c = 0; c < 2; ++c) {
            fill<T>(R, l, u, L.faces_odd, 1 << (c ^ 1));
            R.pre(l, kStageGS);
            HIPCHK(launch_gs<T>(R.s, u, f, lvl_beta<T>(H, l), lvl_faces<T>(H, l), L.d_rb.p, L.wcol.p, L.nwcol, L.ncol,
                                h2, c));
            R.post(l, kStageGS);
        }
}

template <class T>
void bottom(Run& R, size_t l) {
    Hier* H = R.H;
    const Level& L = *H->L[l];
    HIPCHK(launch_bottom<T>(R.s, lvl_u<T>(H, l), lvl_f<T>(H, l), lvl_faces<T>(H, l), H->var && l > 0, L.d_rb.p,
                            (int)L.boxes.size(), L.dom.lo, L.dom.hi, H->per, L.h, R.bottom_rtol, H->iters.p));
}

template <class T>
void vcycle(Run& R, size_t l) {
    Hier* H = R.H;
    const size_t last = H->L.size() - 1;
    if (l == last) {
        bottom<T>(R, l);
        return;
    }
    const Level& L = *H->L[l];
    const Level& C = *H->L[l + 1];
    T* u = lvl_u<T>(H, l);
    smooth<T>(R, l, R.nu1);
    fill<T>(R, l, u, L.faces_odd, 3);
    const T ih2 = (T)(1.0 / (L.h * L.h));
    R.pre(l, kStageRestrict);
    HIPCHK(launch_resid_restrict<T>(R.s, u, lvl_f<T>(H, l), lvl_beta<T>(H, l), lvl_faces<T>(H, l), L.d_rb.p, C.d_rb.p,
                                    L.wdown.p, L.nwdown, L.ndown, ih2, lvl_f<T>(H, l + 1)));
    R.post(l, kStageRestrict);
    HIPCHK(launch_zero<T>(R.s, lvl_u<T>(H, l + 1), C.nelem));
    vcycle<T>(R, l + 1);
    fill<T>(R, l + 1, lvl_u<T>(H, l + 1), C.full_odd, 3);
    R.pre(l, kStageProlong);
    HIPCHK(launch_prolong<T>(R.s, lvl_u<T>(H, l + 1), u, L.d_rb.p, C.d_rb.p, L.wdown.p, L.nwdown, L.ndown, R.prolong));
    R.post(l, kStageProlong);
    smooth<T>(R, l, R.nu2);
}

// Coefficient setup: cell beta at level 0 (exchange + even reflection), then
// face arrays level by level.
template <class T>
void setup_faces(Run& R, T* beta0) {
    Hier* H = R.H;
    const Level& L0 = *H->L[0];
    fill<T>(R, 0, beta0, L0.full_even, 3);
    for (size_t l = 1; l < H->L.size(); ++l) {
        FaceArrays<T> out = lvl_faces<T>(H, l);
        for (int d = 0; d < 3; ++d) {
            T* dst = const_cast<T*>(out.c[d]);
            if (l == 1) {
                HIPCHK(launch_faces_from_cells<T>(R.s, beta0, L0.d_rb.p, L0.wface[d].p, (int)L0.boxes.size(),
                                                  L0.nface[d], d, out, dst));
            } else {
                HIPCHK(launch_faces_coarsen<T>(R.s, lvl_faces<T>(H, l - 1), out, d, dst));
            }
        }
    }
}

double norm_readback(Run& R, double* h_norm, const double* dev) {
    HIPCHK(hipMemcpyAsync(h_norm, dev, 3 * sizeof(double), hipMemcpyDeviceToHost, R.s));
    HIPCHK(hipStreamSynchronize(R.s));
    return h_norm[0];
}

}  // namespace

// ================================================================== C ABI
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
    if (hipHostMalloc((void**)&c->h_norm, 8 * sizeof(double)) != hipSuccess) {
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
    if (ctx->h_norm) (void)hipHostFree(ctx->h_norm);
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
            if (hipMalloc(&mf->data, std::max<size_t>(mf->bytes, 256)) != hipSuccess) return fail(BXMG_ENOMEM, "alloc_multifab: hipMalloc failed");
            mf->owned = true;
        }
        mf->d_fboxes.upload(mf->fboxes);
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

void bxmg_multifab_release(bxmg_multifab mf) {
    if (!mf) return;
    (void)hipSetDevice(mf->ctx->device);
    if (mf->owned) {
        (void)hipStreamSynchronize(mf->ctx->stream);
        (void)hipFree(mf->data);
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
                               ncomp));
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
}

static bxmg_status set_status(bxmg_solve_info* info, bxmg_status st) {
    info->status = st;
    return st;
}

static bxmg_status check_solve_mf(bxmg_multifab m, const bxmg_ba_s* ba, const char* name) {
    if (!m) return fail(BXMG_EINVAL, std::string("solve: ") + name + " is NULL");
    if (m->ba != ba && (m->ba->boxes.size() != ba->boxes.size() ||
                        std::memcmp(m->ba->boxes.data(), ba->boxes.data(), ba->boxes.size() * sizeof(Box)) != 0))
        return fail(BXMG_EINVAL, std::string("solve: ") + name + " is on a different BoxArray");
    if (m->dtype != BXMG_F64) return fail(BXMG_EINVAL, std::string("solve: ") + name + " must be FP64");
    if (m->ng < 1) return fail(BXMG_EINVAL, std::string("solve: ") + name + " needs nghost >= 1");
    return BXMG_OK;
}

static bool covers_domain(const bxmg_ba_s* ba) {
    long long n = 0;
    for (auto& b : ba->boxes) n += b.cells();
    return n == ba->dom.cells();  // boxes are disjoint and inside the domain
}

// The bottom kernel keeps the level's vectors in LDS: at most kMaxBottomCells
// cells and kBottomGrown cells including the ghost layer.
constexpr long long kBottomGrown = 6144;
static bool bottom_fits(const Box& dom) {
    const long long grown = (long long)(dom.n(0) + 2) * (dom.n(1) + 2) * (dom.n(2) + 2);
    return dom.cells() <= kMaxBottomCells && grown <= kBottomGrown;
}

static Hier* get_hier(bxmg_ctx ctx, const bxmg_ba_s* ba, int precision, bool var, double h, bxmg_status* st) {
    char key[128];
    std::snprintf(key, sizeof key, "%llu/%d/%d/%.17g", (unsigned long long)ba->id, precision, (int)var, h);
    auto it = ctx->cache.find(key);
    if (it != ctx->cache.end()) return it->second.get();
    auto lb = make_hierarchy(ba->dom, ba->boxes);
    const LevelBoxes& bot = lb.back();
    if (!bottom_fits(bot.dom)) {
        *st = fail(BXMG_EINVAL, "solve: bottom level has " + std::to_string(bot.dom.cells()) +
                                    " cells (at most 4096, and 6144 with its ghost layer)");
        return nullptr;
    }
    auto H = build_hier(ba, precision, var, h);
    Hier* raw = H.get();
    ctx->cache[key] = std::move(H);
    return raw;
}

bxmg_status bxmg_mlmg_solve(bxmg_ctx ctx, const bxmg_solve_params* params, bxmg_multifab phi, bxmg_multifab rhs,
                            bxmg_multifab beta, bxmg_solve_info* info) {
    if (!ctx || !phi || !rhs || !info) return fail(BXMG_EINVAL, "solve: NULL argument");
    std::memset(info, 0, sizeof(*info));
    bxmg_solve_params P;
    if (params) P = *params;
    else bxmg_solve_params_default(&P);
    const bxmg_ba_s* ba = phi->ba;
    bxmg_status st;
    if ((st = check_solve_mf(phi, ba, "phi")) != BXMG_OK) return set_status(info, st);
    if ((st = check_solve_mf(rhs, ba, "rhs")) != BXMG_OK) return set_status(info, st);
    if (beta && (st = check_solve_mf(beta, ba, "beta")) != BXMG_OK) return set_status(info, st);
    if (!covers_domain(ba)) return set_status(info, fail(BXMG_EINVAL, "solve: the BoxArray must cover its domain"));
    if (P.nu1 < 0 || P.nu2 < 0 || P.max_cycles < 0 || (P.precision != 0 && P.precision != 1) ||
        (P.prolong != 1 && P.prolong != 2))
        return set_status(info, fail(BXMG_EINVAL, "solve: bad parameters"));
    const double h = (P.dx > 0) ? P.dx : 1.0 / ba->dom.n(0);
    std::lock_guard<std::mutex> lock(ctx->mu);
    const auto t0 = std::chrono::steady_clock::now();
    try {
        HIPCHK(hipSetDevice(ctx->device));
        st = BXMG_OK;
        Hier* H = get_hier(ctx, ba, P.precision, beta != nullptr, h, &st);
        if (!H) return set_status(info, st);
        info->levels = (int)H->L.size();
        Run R{H, ctx->stream, P.nu1, P.nu2, P.prolong, P.bottom_rtol};
        R.prof = &ctx->prof;
        const Level& L0 = *H->L[0];
        double* u = H->u64[0]->p;
        double* f = H->f64[0]->p;
        // caller layout -> colour-split level 0
        HIPCHK(launch_fab_to_rb(R.s, (const double*)phi->data, phi->d_fboxes.p, u, false, L0.d_rb.p, L0.wcol.p, L0.nwcol, L0.ncol));
        HIPCHK(launch_fab_to_rb(R.s, (const double*)rhs->data, rhs->d_fboxes.p, f, false, L0.d_rb.p, L0.wcol.p, L0.nwcol, L0.ncol));
        if (beta) {
            HIPCHK(launch_fab_to_rb(R.s, (const double*)beta->data, beta->d_fboxes.p, H->beta64.p, false, L0.d_rb.p, L0.wcol.p, L0.nwcol, L0.ncol));
            if (P.precision == 0) {
                setup_faces<double>(R, H->beta64.p);
            } else {
                fill<double>(R, 0, H->beta64.p, L0.full_even, 3);
                HIPCHK(launch_cast_f32(R.s, H->beta64.p, H->beta32.p, L0.nelem));
                setup_faces<float>(R, H->beta32.p);
            }
        }
        const double ih2 = 1.0 / (L0.h * L0.h);
        const FaceArrays<double> nf = no_faces<double>();
        HIPCHK(launch_field_norm(R.s, f, L0.d_rb.p, L0.wcol.p, L0.nwcol, L0.ncol, H->partials.p, kNormBlocks));
        HIPCHK(launch_norm_final(R.s, H->partials.p, kNormBlocks, H->fnorm.p));
        norm_readback(R, ctx->h_norm, H->fnorm.p);
        const double fnorm = ctx->h_norm[0];
        info->f_inf = fnorm;
        if (ctx->h_norm[2] > 0) {
            info->f_inf = NAN;
            return set_status(info, fail(BXMG_ENONFINITE, "solve: non-finite right-hand side"));
        }
        int status = BXMG_OK;
        int cyc = 0;
        if (fnorm > 0.0) {
            for (;; ++cyc) {
                fill<double>(R, 0, u, L0.faces_odd, 3);
                R.pre(0, kStageResid);
                if (P.precision == 0) {
                    HIPCHK(launch_resid_norm<double>(R.s, u, f, beta ? H->beta64.p : nullptr, nf, L0.d_rb.p, L0.wcol.p,
                                                     L0.nwcol, L0.ncol, ih2, nullptr, H->partials.p, kNormBlocks));
                } else {
                    HIPCHK(launch_resid_cast(R.s, u, f, beta ? H->beta64.p : nullptr, nf, L0.d_rb.p, L0.wcol.p,
                                             L0.nwcol, L0.ncol, ih2, H->f32[0]->p, H->partials.p, kNormBlocks));
                }
                R.post(0, kStageResid);
                HIPCHK(launch_norm_final(R.s, H->partials.p, kNormBlocks, H->fnorm.p));
                norm_readback(R, ctx->h_norm, H->fnorm.p);
                const double rinf = ctx->h_norm[2] > 0 ? NAN : ctx->h_norm[0];
                if (cyc < 256) {
                    info->hist[cyc] = rinf / fnorm;
                    info->hist_l2[cyc] = std::sqrt(ctx->h_norm[1]);
                    info->nhist = cyc + 1;
                }
                info->rel_resid_inf = rinf / fnorm;
                info->resid_l2 = std::sqrt(ctx->h_norm[1]);
                if (!std::isfinite(rinf)) { status = BXMG_ENONFINITE; break; }
                if (P.fixed_cycles > 0) {
                    if (cyc == P.fixed_cycles) break;
                } else {
                    if (rinf <= P.rel_tol * fnorm || rinf <= P.abs_tol) break;
                    if (cyc == P.max_cycles) { status = BXMG_ENOCONV; break; }
                }
                if (P.precision == 0) {
                    vcycle<double>(R, 0);
                } else {
                    HIPCHK(launch_zero<float>(R.s, H->u32[0]->p, L0.nelem));
                    vcycle<float>(R, 0);
                    HIPCHK(launch_add_f32(R.s, u, H->u32[0]->p, L0.d_rb.p, L0.wcol.p, L0.nwcol, L0.ncol));
                }
            }
        }
        info->cycles = cyc;
        if (ba->per[0] && ba->per[1] && ba->per[2])
            HIPCHK(launch_mean_sub(R.s, u, L0.d_rb.p, L0.wcol.p, L0.nwcol, L0.ncol, H->partials.p, kNormBlocks));
        HIPCHK(launch_rb_to_fab(R.s, u, L0.d_rb.p, (double*)phi->data, phi->d_fboxes.p, L0.wcol.p, L0.nwcol, L0.ncol));
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


bxmg_status bxmg_profile_stage(bxmg_ctx ctx, int32_t stage) {
    if (!ctx) return fail(BXMG_EINVAL, "profile_stage: NULL context");
    if (stage < -1 || stage > kStageFill) return fail(BXMG_EINVAL, "profile_stage: unknown stage");
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
    Hier* H = get_hier(ctx, phi->ba, 0, beta != nullptr, h, &st);
    if (!H) return st;
    *Hout = H;
    return BXMG_OK;
}

static void stage_load(Run& R, Hier* H, bxmg_multifab phi, bxmg_multifab rhs, bxmg_multifab beta) {
    const Level& L0 = *H->L[0];
    HIPCHK(launch_fab_to_rb(R.s, (const double*)phi->data, phi->d_fboxes.p, H->u64[0]->p, false, L0.d_rb.p, L0.wcol.p, L0.nwcol, L0.ncol));
    if (rhs) HIPCHK(launch_fab_to_rb(R.s, (const double*)rhs->data, rhs->d_fboxes.p, H->f64[0]->p, false, L0.d_rb.p, L0.wcol.p, L0.nwcol, L0.ncol));
    if (beta) {
        HIPCHK(launch_fab_to_rb(R.s, (const double*)beta->data, beta->d_fboxes.p, H->beta64.p, false, L0.d_rb.p, L0.wcol.p, L0.nwcol, L0.ncol));
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
        fill<double>(R, 0, H->u64[0]->p, L0.faces_odd, 1 << (colour ^ 1));
        HIPCHK(launch_gs<double>(R.s, H->u64[0]->p, H->f64[0]->p, beta ? H->beta64.p : nullptr, no_faces<double>(),
                                 L0.d_rb.p, L0.wcol.p, L0.nwcol, L0.ncol, L0.h * L0.h, colour));
        HIPCHK(launch_rb_to_fab(R.s, H->u64[0]->p, L0.d_rb.p, (double*)phi->data, phi->d_fboxes.p, L0.wcol.p, L0.nwcol, L0.ncol));
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
        fill<double>(R, 0, H->u64[0]->p, L0.faces_odd, 3);
        // r overwrites f in place (each cell reads its own f, then stores r)
        HIPCHK(launch_resid_norm<double>(R.s, H->u64[0]->p, H->f64[0]->p, beta ? H->beta64.p : nullptr,
                                         no_faces<double>(), L0.d_rb.p, L0.wcol.p, L0.nwcol, L0.ncol,
                                         1.0 / (L0.h * L0.h), H->f64[0]->p, H->partials.p, kNormBlocks));
        HIPCHK(launch_norm_final(R.s, H->partials.p, kNormBlocks, H->fnorm.p));
        HIPCHK(launch_rb_to_fab(R.s, H->f64[0]->p, L0.d_rb.p, (double*)r->data, r->d_fboxes.p, L0.wcol.p, L0.nwcol, L0.ncol));
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
        HIPCHK(launch_fab_to_rb(R.s, (const double*)fine->data, fine->d_fboxes.p, H->u64[0]->p, false, L0.d_rb.p, L0.wcol.p, L0.nwcol, L0.ncol));
        HIPCHK(launch_restrict_plain<double>(R.s, H->u64[0]->p, H->f64[1]->p, L0.d_rb.p, L1.d_rb.p, L0.wdown.p, L0.nwdown, L0.ndown));
        HIPCHK(launch_rb_to_fab(R.s, H->f64[1]->p, L1.d_rb.p, (double*)coarse->data, coarse->d_fboxes.p, L1.wcol.p, L1.nwcol, L1.ncol));
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
        HIPCHK(launch_fab_to_rb(R.s, (const double*)fine->data, fine->d_fboxes.p, H->u64[0]->p, false, L0.d_rb.p, L0.wcol.p, L0.nwcol, L0.ncol));
        HIPCHK(launch_fab_to_rb(R.s, (const double*)coarse->data, coarse->d_fboxes.p, H->u64[1]->p, false, L1.d_rb.p, L1.wcol.p, L1.nwcol, L1.ncol));
        fill<double>(R, 1, H->u64[1]->p, L1.full_odd, 3);
        HIPCHK(launch_prolong<double>(R.s, H->u64[1]->p, H->u64[0]->p, L0.d_rb.p, L1.d_rb.p, L0.wdown.p, L0.nwdown, L0.ndown, order));
        HIPCHK(launch_rb_to_fab(R.s, H->u64[0]->p, L0.d_rb.p, (double*)fine->data, fine->d_fboxes.p, L0.wcol.p, L0.nwcol, L0.ncol));
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
        HIPCHK(launch_fab_to_rb(R.s, (const double*)rhs->data, rhs->d_fboxes.p, H->f64[0]->p, false, L0.d_rb.p, L0.wcol.p, L0.nwcol, L0.ncol));
        HIPCHK(launch_bottom<double>(R.s, H->u64[0]->p, H->f64[0]->p, no_faces<double>(), false, L0.d_rb.p,
                                     (int)L0.boxes.size(), L0.dom.lo, L0.dom.hi, H->per, L0.h, rtol, H->iters.p));
        HIPCHK(launch_rb_to_fab(R.s, H->u64[0]->p, L0.d_rb.p, (double*)phi->data, phi->d_fboxes.p, L0.wcol.p, L0.nwcol, L0.ncol));
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
