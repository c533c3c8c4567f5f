// Host-side building blocks shared by the single-problem driver
// (bxmg_host.cpp) and the batch engine (bxmg_batch.cpp): errors, box
// algebra, the level hierarchy, ghost-copy plans, tiles, the colour-split
// layout, device buffers, and the public handle types.  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <deque>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/bxmg.h"
#include "bxmg_internal.h"


// ------------------------------------------------------------------ errors
extern thread_local std::string g_err;  // defined in bxmg_host.cpp

inline bxmg_status fail(bxmg_status st, const std::string& msg) {
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
namespace bxmg {

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

inline Box intersect(const Box& a, const Box& b) {
    Box c;
    for (int d = 0; d < 3; ++d) { c.lo[d] = std::max(a.lo[d], b.lo[d]); c.hi[d] = std::min(a.hi[d], b.hi[d]); }
    return c;
}

inline int floor2(int a) { return a >> 1; }  // arithmetic shift: floor(a/2)

inline Box coarsen(const Box& b) {
    Box c;
    for (int d = 0; d < 3; ++d) { c.lo[d] = floor2(b.lo[d]); c.hi[d] = floor2(b.hi[d]); }
    return c;
}

inline std::vector<std::pair<int, int>> chop1(int lo, int n, int max_box) {
    int bf = 1;
    while (n % (bf * 2) == 0 && bf * 2 <= max_box) bf *= 2;
    const int piece = (max_box / bf) * bf;
    std::vector<std::pair<int, int>> out;
    for (int s = 0; s < n; s += piece) out.push_back({lo + s, lo + std::min(s + piece, n) - 1});
    return out;
}

inline bool domain_coarsenable(const Box& dom) {
    for (int d = 0; d < 3; ++d)
        if (dom.n(d) % 2 || dom.n(d) < 4 || (dom.lo[d] & 1)) return false;
    return true;
}

// Every box holds whole pairs of cells (even lower corner, even edges), so
// each coarse cell's 8 children lie in one box.
inline bool boxes_pair_aligned(const std::vector<Box>& bs) {
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

inline bool boxes_coarsenable(const std::vector<Box>& bs) {
    for (auto& b : bs)
        for (int d = 0; d < 3; ++d)
            if (b.n(d) % 2 || b.n(d) < kMinBoxCoarsen || (b.lo[d] & 1)) return false;
    return true;
}

struct LevelBoxes {
    Box dom;
    std::vector<Box> boxes;
};

inline std::vector<LevelBoxes> make_hierarchy(const Box& dom, const std::vector<Box>& b0) {
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

// The boxes a level runs on (its storage and launches).  Level 0 keeps the
// caller's boxes unless fine_too (solves, which reach the caller's boxes
// through per-box views of the merged storage).  A level whose boxes tile its
// whole domain runs as
// the one domain box, up to kMergeCells cells: the smoother, transfers and
// residuals give the same values under any decomposition (every ghost a
// kernel reads holds exactly the neighbour's value), and one large box has no
// exchange between boxes, long rows and fewer ghost cells.  The logical
// hierarchy (make_hierarchy) is unchanged.
constexpr long long kMergeCells = 1LL << 27;

inline std::vector<Box> execution_boxes(const LevelBoxes& lv, size_t l, bool fine_too = false) {
    if ((l == 0 && !fine_too) || lv.boxes.size() <= 1 || lv.dom.cells() > kMergeCells) return lv.boxes;
    long long vol = 0;
    for (auto& b : lv.boxes) {
        if (!lv.dom.contains(b)) return lv.boxes;
        vol += b.cells();
    }
    if (vol != lv.dom.cells()) return lv.boxes;  // boxes are disjoint: equal volume = exact tiling
    return {lv.dom};
}

// --------------------------------------------------------- ghost-copy plans
// Region tags for the ghost cells of every box grown by ng.
// mode 0: FillBoundary (periodic shifts; ghosts outside a non-periodic face
//         are skipped);  mode 1: physical ghosts only (reflection into the
//         box's own grown data);  mode 2: FillBoundary and physical ghosts in
//         one plan (reflection + shift, read straight from the owning box).
// odd: sign -1 per reflected direction (homogeneous Dirichlet) or +1.
inline std::vector<Tag> build_tags(const Box& dom, const int per[3], const std::vector<Box>& boxes, int ng, bool cross,
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

inline long long tag_cells(const std::vector<Tag>& t) {
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

inline int ilog2ceil(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// Tiles a level launch should have at least (8 per compute unit of the
// 256) before threads walk several planes each.
constexpr long long kMinLevelTiles = 2048;

// min_tiles > 0: walk fewer planes per thread than zc_target where the
// launch would otherwise have fewer than min_tiles tiles (small levels are
// latency-bound: more, shallower threads finish sooner).
inline TileSet make_tiles(const std::vector<std::array<int, 3>>& ext, int zc_target, int ly_cap = 8,
                          long long min_tiles = 0) {
    int mx = 1, my = 1, mz = 1;
    for (auto& e : ext) { mx = std::max(mx, e[0]); my = std::max(my, e[1]); mz = std::max(mz, e[2]); }
    if (mx > 65535 || my > 65535 || mz > 65535) throw std::runtime_error("a box edge exceeds 65535 cells");
    TileSet t;
    t.sh.lx = std::min(ilog2ceil(mx), 6);
    t.sh.ly = std::min(std::min(ilog2ceil(my), 8 - t.sh.lx), std::max(ly_cap, 0));
    t.sh.lz = 8 - t.sh.lx - t.sh.ly;
    const int TX = 1 << t.sh.lx, TY = 1 << t.sh.ly, TZ = 1 << t.sh.lz;
    t.sh.zc = std::max(1, std::min(zc_target, (mz + TZ - 1) / TZ));
    auto count = [&](int zc) {
        long long n = 0;
        for (auto& e : ext)
            n += (long long)((e[0] + TX - 1) / TX) * ((e[1] + TY - 1) / TY) * ((e[2] + TZ * zc - 1) / (TZ * zc));
        return n;
    };
    while (t.sh.zc > 1 && count(t.sh.zc) < min_tiles) t.sh.zc = std::max(1, t.sh.zc / 2);
    const int KZ = TZ * t.sh.zc;
    for (size_t b = 0; b < ext.size(); ++b)
        for (int z0 = 0; z0 < ext[b][2]; z0 += KZ)
            for (int y0 = 0; y0 < ext[b][1]; y0 += TY)
                for (int x0 = 0; x0 < ext[b][0]; x0 += TX) {
                    Tile tl;
                    tl.box = (int)b;
                    tl.x0 = (uint16_t)x0;
                    tl.y0 = (uint16_t)y0;
                    tl.z0 = (uint16_t)z0;
                    tl.lx = (uint8_t)t.sh.lx;
                    tl.ly = (uint8_t)t.sh.ly;
                    tl.lz = (uint8_t)t.sh.lz;
                    tl.zc = (uint8_t)t.sh.zc;
                    tl.pad = 0;
                    t.tiles.push_back(tl);
                }
    return t;
}

// The colour-cell tiles of a level: zc planes per thread, or zc_planes where
// a tile spans whole box planes.
inline TileSet level_tiles(const std::vector<std::array<int, 3>>& ecol, int zc, int zc_planes, int ly_cap,
                           long long min_tiles) {
    TileSet ts = make_tiles(ecol, zc, ly_cap, min_tiles);
    if (ts.sh.lz == 0) ts = make_tiles(ecol, zc_planes, ly_cap, min_tiles);
    return ts;
}

// Upper bound of the coarse values a tile of this shape reads in a
// prolongation (parents of its cells and one layer around them; the fine
// boxes are pair aligned): what the LDS-staged kernel must hold.
inline int prolong_stage_values(const TileShape& sh) {
    const int TX = 1 << sh.lx, TY = 1 << sh.ly, TZ = (1 << sh.lz) * sh.zc;
    return (TX + 3) * (((TY + 1) >> 1) + 3) * (((TZ + 1) >> 1) + 3);
}

// The tiles over which the periodic solution mean is summed: a fixed shape
// that no launch knob changes, so the mean's rounding -- and with it every
// bit of a periodic solution -- does not depend on the knobs; the lone and
// the batched solve both use it.
inline TileSet mean_tiles(const std::vector<std::array<int, 3>>& ecol) { return level_tiles(ecol, 4, 4, 8, 0); }

// Colour-cell extents: ceil(nx/2) cells of one colour per row.
inline std::vector<std::array<int, 3>> colour_extents(const std::vector<Box>& boxes) {
    std::vector<std::array<int, 3>> e;
    for (auto& b : boxes) e.push_back({(b.n(0) + 1) / 2, b.n(1), b.n(2)});
    return e;
}

// Coarse-cell extents of every fine box; extra_d >= 0 adds the high face
// layer in direction d for boxes touching the fine domain's upper end.
inline std::vector<std::array<int, 3>> coarse_extents(const std::vector<Box>& fine, const Box& fdom, int extra_d) {
    std::vector<std::array<int, 3>> e;
    for (auto& b : fine) {
        std::array<int, 3> x{b.n(0) / 2, b.n(1) / 2, b.n(2) / 2};
        if (extra_d >= 0 && b.hi[extra_d] == fdom.hi[extra_d]) x[extra_d] += 1;
        e.push_back(x);
    }
    return e;
}

inline std::vector<int> coarse_owner(const std::vector<Box>& fine, const std::vector<Box>& coarse) {
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
inline std::vector<RBox> rb_layout(const std::vector<Box>& boxes, int ng, double h, long long* nelem) {
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
        r.h = h;
        r.a = 0.0;
        for (int q = 0; q < 6; ++q) { r.nb[q] = -2; r.shift[q] = 0; }
        const long long half = (long long)r.H * r.G[1] * r.G[2];
        const long long padded = (half + 63) / 64 * 64;
        if (2 * padded > 0x7fffffffLL) throw std::runtime_error("a box holds more than 2^31 elements");
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
inline bool face_neighbours(const Box& dom, const int per[3], const std::vector<Box>& boxes, std::vector<RBox>& rb) {
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

// Boxes small enough for 32-bit buffer addressing of both colour blocks
// in FP64 (byte offsets and the descriptor's record count are 32-bit).
inline bool boxes_fit_res(const std::vector<RBox>& rb) {
    for (auto& r : rb)
        if (2 * r.cstride * 8 >= 0x7fffffffLL) return false;
    return true;
}

inline long long rb_index(const RBox& b, int i, int j, int k) {
    return b.base + (long long)((i + j + k) & 1) * b.cstride +
           ((long long)(k - b.glo[2]) * b.G[1] + (j - b.glo[1])) * b.H + ((i - b.glo[0]) >> 1);
}

// Expand region tags into per-cell (dst, src) element pairs of an RB level,
// keeping the destinations whose colour is in cmask.
inline std::vector<GhostCopy> ghost_list(const std::vector<Tag>& tags, const std::vector<RBox>& rb, int cmask) {
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
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            if (p) (void)hipFree(p);
            p = o.p;
            n = o.n;
            o.p = nullptr;
            o.n = 0;
        }
        return *this;
    }
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
    // From the stream-ordered allocator on stream s; the stream is drained
    // before returning, so the memory is ready for work on any stream.
    void upload_async(const std::vector<T>& v, hipStream_t s) {
        if (p) { (void)hipFree(p); p = nullptr; }
        n = v.size();
        if (v.empty()) return;
        HIPCHK(hipMallocAsync((void**)&p, v.size() * sizeof(T), s));
        HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    // Stream-ordered free on s: after the work queued there so far.
    void release_async(hipStream_t s) {
        if (p) (void)hipFreeAsync(p, s);
        p = nullptr;
        n = 0;
    }
};

// Device array that keeps its allocation and only grows (no free on refill).
template <class T>
struct DevVec {
    DevBuf<T> b;
    size_t len = 0;
    T* p() const { return b.p; }
    void reserve(size_t count) {
        if (count > b.n) b.alloc(std::max<size_t>(count, b.n + b.n / 2));
    }
    void assign(const std::vector<T>& v) {
        reserve(std::max<size_t>(v.size(), 1));
        len = v.size();
        if (!v.empty()) HIPCHK(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    }
};

// For every block of kBlock region cells, the tag of its first cell; then
// ntags - 1.  The fill and copy kernels search only between a block's two
// entries.
inline std::vector<int> tag_hints(const std::vector<Tag>& t) {
    std::vector<int> h;
    if (t.empty()) return h;
    const long long cells = tag_cells(t);
    size_t q = 0;
    for (long long g = 0; g < cells; g += kBlock) {
        while (q + 1 < t.size() && t[q + 1].prefix <= g) ++q;
        h.push_back((int)q);
    }
    h.push_back((int)t.size() - 1);
    return h;
}

struct Plan {
    DevBuf<Tag> tags;
    DevBuf<int> hints;
    int ntags = 0;
    long long cells = 0;
    void set(const std::vector<Tag>& t, hipStream_t s) {
        tags.upload_async(t, s);
        hints.upload_async(tag_hints(t), s);
        ntags = (int)t.size();
        cells = tag_cells(t);
    }
};

}  // namespace bxmg

using namespace bxmg;

// ============================================================ public handles
struct bxmg_ba_s {
    Box dom;
    int bc[3];
    int per[3];
    std::vector<Box> boxes;
    std::atomic<int> refs{1};
    uint64_t id;
};

extern std::atomic<uint64_t> g_next_id;  // defined in bxmg_host.cpp

inline void ba_release(bxmg_ba_s* ba) {
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
    int res = 1;                // 32-bit buffer addressing where the boxes allow it
    int ly_cap = 8;             // at most 2^ly_cap threads of a tile along y
    int lds_coarse = 1;         // fused coarse cycle keeps its levels in LDS when they fit
    int merge = 1;              // solves run levels that tile their domain as one box
    std::map<std::string, std::unique_ptr<Hier>> cache;  // by geometry and settings
    std::deque<std::string> lru;                          // cache keys, least recently used first
    double* h_norm = nullptr;  // pinned
    void* h_solve = nullptr;   // pinned: a solve's stop-test state read back (history, slot, flag)
    void* scratch = nullptr;   // the device's staging array (scratch_address), kScratchBytes
    std::shared_ptr<void> nodal;  // nodal-solver hierarchies (bxmg_nodal.hip)
    std::shared_ptr<void> composite;  // composite-solve state of the last layout (bxmg_composite.hip)
    std::mutex comp_mu;               // composite solves on one context run one at a time
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
    // region lists kept on the host only, staged per call (allocation-free calls)
    std::map<int, std::pair<std::vector<Tag>, long long>> host_plans;
    // ParallelCopy plans into this MultiFab, by (source BoxArray id, copy width)
    std::map<std::pair<uint64_t, int>, std::unique_ptr<Plan>> pcopy_plans;
};

// ParallelCopy regions: every box of dst grown by ngc, against every
// source box and its periodic images (shifts of the domain edge in the
// periodic directions); a region's source cell is its cell + soff.  With
// ngc <= the domain edge in periodic directions each destination cell has
// at most one image in the source's (disjoint) valid regions.
inline std::vector<Tag> pcopy_tags(const Box& dom, const int per[3], const std::vector<Box>& dst, int ngc,
                                   const std::vector<Box>& src) {
    std::vector<Tag> tags;
    long long prefix = 0;
    for (size_t b = 0; b < dst.size(); ++b) {
        Box G = dst[b];
        for (int d = 0; d < 3; ++d) { G.lo[d] -= ngc; G.hi[d] += ngc; }
        for (int sz = -1; sz <= 1; ++sz)
            for (int sy = -1; sy <= 1; ++sy)
                for (int sx = -1; sx <= 1; ++sx) {
                    const int sh[3] = {sx, sy, sz};
                    bool skip = false;
                    for (int d = 0; d < 3; ++d)
                        if (sh[d] && !per[d]) skip = true;
                    if (skip) continue;
                    for (size_t o = 0; o < src.size(); ++o) {
                        Box S = src[o];
                        for (int d = 0; d < 3; ++d) { S.lo[d] += sh[d] * dom.n(d); S.hi[d] += sh[d] * dom.n(d); }
                        const Box I = intersect(G, S);
                        if (!I.ok()) continue;
                        Tag t;
                        std::memset(&t, 0, sizeof t);
                        t.dbox = (int)b;
                        t.sbox = (int)o;
                        for (int d = 0; d < 3; ++d) {
                            t.dlo[d] = I.lo[d];
                            t.n[d] = I.n(d);
                            t.soff[d] = -sh[d] * dom.n(d);
                            t.sgn[d] = 1;
                        }
                        t.neg = 0;
                        t.prefix = prefix;
                        prefix += I.cells();
                        tags.push_back(t);
                    }
                }
    }
    return tags;
}

inline size_t mf_layout(const bxmg_ba_s* ba, int ncomp, int ng, bxmg_dtype dt, std::vector<FBox>* out) {
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

inline Plan* mf_plan(bxmg_mf_s* mf, int mode, bool cross, bool odd) {
    const int key = mode * 4 + (cross ? 2 : 0) + (odd ? 1 : 0);
    auto it = mf->plans.find(key);
    if (it != mf->plans.end()) return it->second.get();
    auto p = std::make_unique<Plan>();
    p->set(build_tags(mf->ba->dom, mf->ba->per, mf->ba->boxes, mf->ng, cross, mode, odd), mf->ctx->stream);
    Plan* raw = p.get();
    mf->plans[key] = std::move(p);
    return raw;
}

// ------------------------------------------------------- solve argument checks
inline bxmg_status check_solve_mf(bxmg_multifab m, const bxmg_ba_s* ba, const char* name) {
    if (!m) return fail(BXMG_EINVAL, std::string("solve: ") + name + " is NULL");
    if (m->ba != ba && (m->ba->boxes.size() != ba->boxes.size() ||
                        std::memcmp(m->ba->boxes.data(), ba->boxes.data(), ba->boxes.size() * sizeof(Box)) != 0))
        return fail(BXMG_EINVAL, std::string("solve: ") + name + " is on a different BoxArray");
    if (m->dtype != BXMG_F64) return fail(BXMG_EINVAL, std::string("solve: ") + name + " must be FP64");
    if (m->ng < 1) return fail(BXMG_EINVAL, std::string("solve: ") + name + " needs nghost >= 1");
    return BXMG_OK;
}

// A field read at valid cells only (a source term): same boxes, FP64, any ghost width
inline bxmg_status check_field_mf(bxmg_multifab m, const bxmg_ba_s* ba, const char* name) {
    if (m->ba != ba && (m->ba->boxes.size() != ba->boxes.size() ||
                        std::memcmp(m->ba->boxes.data(), ba->boxes.data(), ba->boxes.size() * sizeof(Box)) != 0))
        return fail(BXMG_EINVAL, std::string("solve: ") + name + " is on a different BoxArray");
    if (m->dtype != BXMG_F64) return fail(BXMG_EINVAL, std::string("solve: ") + name + " must be FP64");
    return BXMG_OK;
}

inline bool covers_domain(const bxmg_ba_s* ba) {
    long long n = 0;
    for (auto& b : ba->boxes) n += b.cells();
    return n == ba->dom.cells();  // boxes are disjoint and inside the domain
}

// The bottom kernel keeps the level's vectors in LDS: at most kMaxBottomCells
// cells and kBottomGrown cells including the ghost layer.
inline bool bottom_fits(const Box& dom) {
    const long long grown = (long long)(dom.n(0) + 2) * (dom.n(1) + 2) * (dom.n(2) + 2);
    return dom.cells() <= kMaxBottomCells && grown <= kBottomGrown;
}

// An FP64 constant-coefficient Poisson hierarchy of ba owned by the caller
// (not in the context's cache); throws std::runtime_error when its bottom
// level is too large, HipError on device errors.
std::shared_ptr<Hier> hier_create(bxmg_ctx ctx, const bxmg_ba_s* ba, double h);
// Its level-0 colour-split arrays (solution, right-hand side), the layout of
// its single level-0 box, and its depth.
void hier_level0(Hier* H, double** u, double** f, RBox* box, int* levels);
// One V-cycle from zero on the level-0 right-hand side as it stands;
// asynchronous on the context's stream.
void hier_vcycle_from_zero(bxmg_ctx ctx, Hier* H, const bxmg_solve_params& P);

