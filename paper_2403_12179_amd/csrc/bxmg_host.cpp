// Host side of libbxmg: BoxArrays, MultiFabs, cached ghost-copy plans, the
// multigrid hierarchy and the V-cycle driver, behind the C ABI of bxmg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
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

#define HIPCHK(...)                                                   \
    do {                                                              \
        hipError_t e_ = (__VA_ARGS__);                                \
        if (e_ != hipSuccess) throw HipError{e_, #__VA_ARGS__};       \
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

// Every box holds whole pairs of cells (even lower corner, even edges), so
// each coarse cell's 8 children lie in one box.
bool boxes_pair_aligned(const std::vector<Box>& bs) {
    for (auto& b : bs)
        for (int d = 0; d < 3; ++d)
            if (b.n(d) % 2 || (b.lo[d] & 1)) return false;
    return true;
}

// Boxes are coarsened one by one while every box edge is at least
// kMinBoxCoarsen; smaller boxes are merged into one box per level (fewer,
// larger boxes on the coarse levels: less ghost overhead, and the small
// single-box levels can run as one fused coarse cycle).
constexpr int kMinBoxCoarsen = 32;

bool boxes_coarsenable(const std::vector<Box>& bs) {
    for (auto& b : bs)
        for (int d = 0; d < 3; ++d)
            if (b.n(d) % 2 || b.n(d) < kMinBoxCoarsen || (b.lo[d] & 1)) return false;
    return true;
}

struct LevelBoxes {
    Box dom;
    std::vector<Box> boxes;
};

std::vector<LevelBoxes> make_hierarchy(const Box& dom, const std::vector<Box>& b0) {
    std::vector<LevelBoxes> L{LevelBoxes{dom, b0}};
    while (domain_coarsenable(L.back().dom) && boxes_pair_aligned(L.back().boxes)) {
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

// Tiles: one block of kBlock threads per tile, TX x TY x TZ threads with
// TX = 2^lx covering x, TY = 2^ly covering y, TZ = 2^lz planes walked zc
// times.  ext[b] = per-box thread extents (x, y, z).  Tiles run box-major,
// then z, y, x, so consecutive tiles share halo planes.
struct TileSet {
    std::vector<Tile> tiles;
    TileShape sh;
};

int ilog2ceil(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

TileSet make_tiles(const std::vector<std::array<int, 3>>& ext, int zc_target) {
    int mx = 1, my = 1, mz = 1;
    for (auto& e : ext) { mx = std::max(mx, e[0]); my = std::max(my, e[1]); mz = std::max(mz, e[2]); }
    TileSet t;
    t.sh.lx = std::min(ilog2ceil(mx), 6);
    t.sh.ly = std::min(ilog2ceil(my), 8 - t.sh.lx);
    t.sh.lz = 8 - t.sh.lx - t.sh.ly;
    const int TX = 1 << t.sh.lx, TY = 1 << t.sh.ly, TZ = 1 << t.sh.lz;
    t.sh.zc = std::max(1, std::min(zc_target, (mz + TZ - 1) / TZ));
    const int KZ = TZ * t.sh.zc;
    for (size_t b = 0; b < ext.size(); ++b)
        for (int z0 = 0; z0 < ext[b][2]; z0 += KZ)
            for (int y0 = 0; y0 < ext[b][1]; y0 += TY)
                for (int x0 = 0; x0 < ext[b][0]; x0 += TX) t.tiles.push_back(Tile{(int)b, x0, y0, z0});
    return t;
}

// Colour-cell extents: ceil(nx/2) cells of one colour per row.
std::vector<std::array<int, 3>> colour_extents(const std::vector<Box>& boxes) {
    std::vector<std::array<int, 3>> e;
    for (auto& b : boxes) e.push_back({(b.n(0) + 1) / 2, b.n(1), b.n(2)});
    return e;
}

// Coarse-cell extents of every fine box; extra_d >= 0 adds the high face
// layer in direction d for boxes touching the fine domain's upper end.
std::vector<std::array<int, 3>> coarse_extents(const std::vector<Box>& fine, const Box& fdom, int extra_d) {
    std::vector<std::array<int, 3>> e;
    for (auto& b : fine) {
        std::array<int, 3> x{b.n(0) / 2, b.n(1) / 2, b.n(2) / 2};
        if (extra_d >= 0 && b.hi[extra_d] == fdom.hi[extra_d]) x[extra_d] += 1;
        e.push_back(x);
    }
    return e;
}

std::vector<int> coarse_owner(const std::vector<Box>& fine, const std::vector<Box>& coarse) {
    std::vector<int> own;
    for (auto& b : fine) {
        const Box c = coarsen(b);
        int o = -1;
        for (size_t q = 0; q < coarse.size(); ++q)
            if (coarse[q].contains(c)) { o = (int)q; break; }
        if (o < 0) throw std::runtime_error("a coarsened box lies in no coarse box");
        own.push_back(o);
    }
    return own;
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
        for (int q = 0; q < 6; ++q) { r.nb[q] = -2; r.shift[q] = 0; }
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

// Face neighbours of every box of a level (RBox::nb / shift).  Returns true
// when each face is resolvable: the 1-cell slab beyond it lies in one box
// (after a periodic shift) or outside a Dirichlet domain face.
bool face_neighbours(const Box& dom, const int per[3], const std::vector<Box>& boxes, std::vector<RBox>& rb) {
    bool all = true;
    for (size_t b = 0; b < boxes.size(); ++b)
        for (int d = 0; d < 3; ++d)
            for (int side = 0; side < 2; ++side) {
                const int q = 2 * d + side;
                Box S = boxes[b];
                S.lo[d] = S.hi[d] = side ? boxes[b].hi[d] + 1 : boxes[b].lo[d] - 1;
                int shift = 0;
                if (S.lo[d] < dom.lo[d] || S.lo[d] > dom.hi[d]) {
                    if (!per[d]) {
                        rb[b].nb[q] = -1;
                        rb[b].shift[q] = 0;
                        continue;
                    }
                    shift = side ? -dom.n(d) : dom.n(d);
                    S.lo[d] += shift;
                    S.hi[d] += shift;
                }
                int found = -2;
                for (size_t o = 0; o < boxes.size(); ++o)
                    if (boxes[o].contains(S)) { found = (int)o; break; }
                rb[b].nb[q] = found;
                rb[b].shift[q] = shift;
                if (found == -2) all = false;
            }
    return all;
}

long long rb_index(const RBox& b, int i, int j, int k) {
    return b.base + (long long)((i + j + k) & 1) * b.cstride +
           ((long long)(k - b.glo[2]) * b.G[1] + (j - b.glo[1])) * b.H + ((i - b.glo[0]) >> 1);
}

// Expand region tags into per-cell (dst, src) element pairs of an RB level,
// keeping the destinations whose colour is in cmask.
std::vector<GhostCopy> ghost_list(const std::vector<Tag>& tags, const std::vector<RBox>& rb, int cmask) {
    std::vector<GhostCopy> out;
    for (auto& t : tags)
        for (int z = 0; z < t.n[2]; ++z)
            for (int y = 0; y < t.n[1]; ++y)
                for (int x = 0; x < t.n[0]; ++x) {
                    const int di = t.dlo[0] + x, dj = t.dlo[1] + y, dk = t.dlo[2] + z;
                    if (!((cmask >> ((di + dj + dk) & 1)) & 1)) continue;
                    const int si = t.sgn[0] * di + t.soff[0], sj = t.sgn[1] * dj + t.soff[1],
                              sk = t.sgn[2] * dk + t.soff[2];
                    const long long d = rb_index(rb[t.dbox], di, dj, dk), sr = rb_index(rb[t.sbox], si, sj, sk);
                    if (d < 0 || sr < 0 || d > 0x7fffffffLL || sr > 0x7fffffffLL)
                        throw std::runtime_error("level storage exceeds 2^31 elements");
                    out.push_back(GhostCopy{(uint32_t)d, (uint32_t)sr | (t.neg ? 0x80000000u : 0u)});
                }
    return out;
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
    int zc = 4, zc_planes = 4;  // tile depths for hierarchies built from now on
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
    TileShape shcol{};
    // transfer tiles to level + 1 (coarse cells of every box)
    DevBuf<Tile> tdown;
    int ntdown = 0;
    TileShape shdown{};
    DevBuf<int> cbox;
    // coefficient setup tiles (coarse faces anchored in every box), level 0
    DevBuf<Tile> tface[3];
    int ntface[3] = {0, 0, 0};
    TileShape shface[3]{};
    GhostList face[2];  // face ghosts of colour c: exchange + Dirichlet
    GhostList full;     // every ghost: exchange + Dirichlet
    GhostList full_even;  // every ghost: exchange + even reflection (cell beta)
    bool push = false;    // producers refresh the face ghosts they mirror
    Grid grid() const { return Grid{d_rb.p, tcol.p, ntcol, shcol, push ? 1 : 0}; }
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
    int coarse_start = -1;    // first level of the fused coarse cycle (-1: none)
    DevBuf<CoarseCycle<double>> cc64;  // device copies of the descriptors ...
    DevBuf<CoarseCycle<float>> cc32;
    CoarseCycle<double> cc64_host{};   // ... and what they hold
    CoarseCycle<float> cc32_host{};
    DevBuf<double> partials;  // 3 per tile of the largest tiled launch, + 3
    DevBuf<double> fnorm;     // 3
    DevBuf<int> iters;
    size_t bytes = 0;
    XGrid xgrid(size_t l) const {
        const Level& F = *L[l];
        const Level& C = *L[l + 1];
        return XGrid{F.d_rb.p, C.d_rb.p, F.cbox.p, F.tdown.p, F.ntdown, F.shdown, F.push ? 1 : 0};
    }
    XGrid face_grid(int d) const {
        const Level& F = *L[0];
        const Level& C = *L[1];
        return XGrid{F.d_rb.p, C.d_rb.p, F.cbox.p, F.tface[d].p, F.ntface[d], F.shface[d], 0};
    }
};

// Tile depth: planes walked per thread in the cell kernels (a tuning knob,
// bxmg_ctx_tune), separately for tiles that span whole box planes.
struct Tuning {
    int zc = 4;
    int zc_planes = 4;
};

static void upload_tiles(const TileSet& t, DevBuf<Tile>& buf, int& n, TileShape& sh) {
    buf.upload(t.tiles);
    n = (int)t.tiles.size();
    sh = t.sh;
}

static std::unique_ptr<Hier> build_hier(const bxmg_ba_s* ba, int precision, bool var, double h0, const Tuning& tune) {
    auto H = std::make_unique<Hier>();
    for (int d = 0; d < 3; ++d) H->per[d] = ba->per[d];
    H->precision = precision;
    H->var = var;
    std::vector<LevelBoxes> lb = make_hierarchy(ba->dom, ba->boxes);
    double h = h0;
    long long max_tiles = 1;
    for (size_t l = 0; l < lb.size(); ++l) {
        auto lv = std::make_unique<Level>();
        lv->dom = lb[l].dom;
        lv->h = h;
        h *= 2.0;
        lv->boxes = lb[l].boxes;
        lv->rb = rb_layout(lv->boxes, 1, &lv->nelem);
        lv->push = face_neighbours(lv->dom, H->per, lv->boxes, lv->rb);
        lv->d_rb.upload(lv->rb);
        {
            TileSet ts = make_tiles(colour_extents(lv->boxes), tune.zc);
            if (ts.sh.lz == 0) ts = make_tiles(colour_extents(lv->boxes), tune.zc_planes);
            upload_tiles(ts, lv->tcol, lv->ntcol, lv->shcol);
        }
        max_tiles = std::max<long long>(max_tiles, lv->ntcol);
        if (l + 1 < lb.size()) {
            upload_tiles(make_tiles(coarse_extents(lv->boxes, lv->dom, -1), tune.zc), lv->tdown, lv->ntdown, lv->shdown);
            lv->cbox.upload(coarse_owner(lv->boxes, lb[l + 1].boxes));
            if (var && l == 0)
                for (int d = 0; d < 3; ++d)
                    upload_tiles(make_tiles(coarse_extents(lv->boxes, lv->dom, d), tune.zc), lv->tface[d], lv->ntface[d],
                                 lv->shface[d]);
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
        }
    }
    H->partials.alloc(3 * max_tiles + 8);
    H->fnorm.alloc(4);
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
    // event brackets around level-0 launches of the profiled stage
    void pre(size_t l, int stage) { if (prof && prof->stage == stage && l == 0) prof->mark(s); }
    void post(size_t l, int stage) { if (prof && prof->stage == stage && l == 0) prof->mark(s); }
};

enum { kStageGS = 0, kStageResid = 1, kStageRestrict = 2, kStageProlong = 3, kStageFill = 4 };

template <class T>
void fill(Run& R, size_t l, T* data, const GhostList& g) {
    R.pre(l, kStageFill);
    HIPCHK(launch_fill_rb(R.s, data, sizeof(T) == 4, g.list.p, g.n));
    R.post(l, kStageFill);
}

// both colours' face ghosts: two lists (the solver refreshes them per colour)
template <class T>
void fill_faces(Run& R, size_t l, T* data) {
    const Level& L = *R.H->L[l];
    fill<T>(R, l, data, L.face[0]);
    fill<T>(R, l, data, L.face[1]);
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
            if (!L.push) fill<T>(R, l, u, L.face[c ^ 1]);
            R.pre(l, kStageGS);
            HIPCHK(launch_gs<T>(R.s, L.grid(), u, f, lvl_beta<T>(H, l), lvl_faces<T>(H, l), h2, c));
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
void coarse_cycle(Run& R) {
    Hier* H = R.H;
    static_assert(std::is_trivially_copyable<CoarseCycle<T>>::value, "descriptor must be plain data");
    DevBuf<CoarseCycle<T>>& buf = cc_buf<T>(H);
    CoarseCycle<T>& host = cc_host<T>(H);
    const CoarseCycle<T> cc = coarse_desc<T>(H, R.nu1, R.nu2, R.prolong, R.bottom_rtol);
    if (!buf.p || std::memcmp(&cc, &host, sizeof cc) != 0) {
        if (!buf.p) buf.alloc(1);
        host = cc;  // lives as long as the hierarchy: safe source for the async copy
        HIPCHK(hipMemcpyAsync(buf.p, &host, sizeof host, hipMemcpyHostToDevice, R.s));
    }
    HIPCHK(launch_coarse_cycle<T>(R.s, buf.p, H->var));
}

template <class T>
void vcycle(Run& R, size_t l) {
    Hier* H = R.H;
    const size_t last = H->L.size() - 1;
    if ((int)l == H->coarse_start) {
        coarse_cycle<T>(R);
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
    const T ih2 = (T)(1.0 / (L.h * L.h));
    R.pre(l, kStageRestrict);
    HIPCHK(launch_resid_restrict<T>(R.s, H->xgrid(l), u, lvl_f<T>(H, l), lvl_beta<T>(H, l), lvl_faces<T>(H, l), ih2,
                                    lvl_f<T>(H, l + 1)));
    R.post(l, kStageRestrict);
    HIPCHK(launch_zero<T>(R.s, lvl_u<T>(H, l + 1), C.nelem));
    vcycle<T>(R, l + 1);
    fill<T>(R, l + 1, lvl_u<T>(H, l + 1), C.full);
    R.pre(l, kStageProlong);
    HIPCHK(launch_prolong<T>(R.s, L.grid(), C.d_rb.p, L.cbox.p, lvl_u<T>(H, l + 1), u, R.prolong));
    R.post(l, kStageProlong);
    smooth<T>(R, l, R.nu2);
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
static bool bottom_fits(const Box& dom) {
    const long long grown = (long long)(dom.n(0) + 2) * (dom.n(1) + 2) * (dom.n(2) + 2);
    return dom.cells() <= kMaxBottomCells && grown <= kBottomGrown;
}

static Hier* get_hier(bxmg_ctx ctx, const bxmg_ba_s* ba, int precision, bool var, double h, bxmg_status* st) {
    char key[128];
    std::snprintf(key, sizeof key, "%llu/%d/%d/%.17g/%d/%d", (unsigned long long)ba->id, precision, (int)var, h,
                  ctx->zc, ctx->zc_planes);
    auto it = ctx->cache.find(key);
    if (it != ctx->cache.end()) return it->second.get();
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
        H = build_hier(ba, precision, var, h, tune);
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
        HIPCHK(launch_fab_to_rb(R.s, L0.grid(), (const double*)phi->data, phi->d_fboxes.p, u, false));
        HIPCHK(launch_fab_to_rb(R.s, L0.grid(), (const double*)rhs->data, rhs->d_fboxes.p, f, false));
        if (beta) {
            HIPCHK(launch_fab_to_rb(R.s, L0.grid(), (const double*)beta->data, beta->d_fboxes.p, H->beta64.p, false));
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
        const double ih2 = 1.0 / (L0.h * L0.h);
        const FaceArrays<double> nf = no_faces<double>();
        HIPCHK(launch_field_norm(R.s, L0.grid(), f, H->partials.p));
        HIPCHK(launch_norm_final(R.s, H->partials.p, L0.ntcol, H->fnorm.p));
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
                if (!L0.push) fill_faces<double>(R, 0, u);
                R.pre(0, kStageResid);
                if (P.precision == 0) {
                    HIPCHK(launch_resid<double, double>(R.s, L0.grid(), u, f, beta ? H->beta64.p : nullptr, nf, ih2,
                                                        (double*)nullptr, H->partials.p));
                } else {
                    HIPCHK(launch_resid<double, float>(R.s, L0.grid(), u, f, beta ? H->beta64.p : nullptr, nf, ih2,
                                                       H->f32[0]->p, H->partials.p));
                }
                R.post(0, kStageResid);
                HIPCHK(launch_norm_final(R.s, H->partials.p, L0.ntcol, H->fnorm.p));
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
                    HIPCHK(launch_add_f32(R.s, L0.grid(), u, H->u32[0]->p));
                }
            }
        }
        info->cycles = cyc;
        if (ba->per[0] && ba->per[1] && ba->per[2])
            HIPCHK(launch_mean_sub(R.s, L0.grid(), u, H->partials.p));
        HIPCHK(launch_rb_to_fab(R.s, L0.grid(), u, (double*)phi->data, phi->d_fboxes.p));
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


bxmg_status bxmg_ctx_tune(bxmg_ctx ctx, int32_t param, int32_t value) {
    if (!ctx) return fail(BXMG_EINVAL, "ctx_tune: NULL context");
    if (value < 1 || value > 64) return fail(BXMG_EINVAL, "ctx_tune: value out of range [1, 64]");
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (param == 0) ctx->zc = value;
    else if (param == 1) ctx->zc_planes = value;
    else return fail(BXMG_EINVAL, "ctx_tune: unknown parameter");
    return BXMG_OK;
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
                                 no_faces<double>(), L0.h * L0.h, colour));
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
                                            no_faces<double>(), 1.0 / (L0.h * L0.h), H->f64[0]->p, H->partials.p));
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
                                     (int)L0.boxes.size(), L0.dom.lo, L0.dom.hi, H->per, L0.h, rtol, H->iters.p));
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
