// Internal declarations shared by the host driver (bxmg_host.cpp) and the
// HIP kernels (bxmg_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bxmg {

constexpr int kMaxBottomCells = 4096;  // bottom level: one workgroup, vectors in LDS
constexpr int kBottomGrown = 6144;     // ... and at most this many cells with its ghost layer
constexpr int kBlock = 256;            // threads per block of the cell kernels

// Block coordinates with consecutive logical blocks on one XCD: blocks are
// dispatched round-robin over the 8 XCDs (block p to XCD p % 8), so logical
// block (p % 8) * (N / 8) + p / 8 gives each XCD one contiguous eighth of the
// grid (x fastest, then y, then z), and its L2 serves the neighbouring rows
// and planes its stencils read.
__device__ __forceinline__ uint3 xcd_block() {
    const unsigned gx = gridDim.x, gy = gridDim.y, N = gx * gy * gridDim.z;
    const unsigned p = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned L = (N & 7) ? p : (p & 7) * (N >> 3) + (p >> 3);
    const unsigned r = L / gx;
    return make_uint3(L - r * gx, r % gy, r / gy);
}

// Box of a level in the multigrid hierarchy, colour-split storage ("RB").
// Cells of colour c = (i+j+k)&1 of the box grown by ng are stored as half
// rows: element (i,j,k) sits at
//   base + c*cstride + ((k-glo.z)*G.y + (j-glo.y))*H + ((i-glo.x)>>1).
// Both colours of a row share the half-row index m = (i-glo.x)>>1.
//
// Face neighbours: for direction q = 2*d + (0 low side, 1 high side), the
// 1-cell slab just outside the box across that face lies in box nb[q] once
// coordinate d is shifted by shift[q] (a periodic image), or, when
// nb[q] == -1, outside a homogeneous-Dirichlet domain face.  Conversely a
// cell of this box on face q is the ghost cell (coordinate d + shift[q]) of
// box nb[q].  nb[q] == -2: not resolvable through one box.
struct RBox {
    int lo[3], hi[3];  // valid cells, global
    int glo[3];        // lo - ng
    int G[3];          // grown extents
    int H;             // half-row pitch = (G.x + 1) / 2
    int pid;           // problem slot (batches); 0 for a single problem
    long long base;    // element offset of colour 0
    long long cstride; // elements between colour 0 and colour 1
    double h;          // grid spacing of the box's level
    double a;          // Helmholtz coefficient alpha: the operator is div(beta grad u) - alpha u
    int nb[6];
    int shift[6];
};

// Box of a caller MultiFab (F-order): element (i,j,k,n) at
//   base + n*cs + (i-glo.x) + G.x*((j-glo.y) + G.y*(k-glo.z)).
struct FBox {
    int lo[3], hi[3];
    int glo[3];
    int G[3];
    long long base;
    long long cs;  // component stride
};

// One rectangular ghost-copy region (caller MultiFabs): destination cells
// dlo + (x,y,z), 0 <= x < n[0] ..., of box dbox take neg ? -v : v, v = the
// cell s_d = sgn_d * dst_d + soff_d of box sbox.  prefix = cells before it.
struct Tag {
    int dbox, sbox;
    int dlo[3];
    int n[3];
    int soff[3];
    int sgn[3];
    int neg;
    int pad;
    long long prefix;
};

// One ghost cell of a level (RB storage): data[dst] = +-data[src & 0x7fffffff],
// negated when bit 31 of src is set.
struct GhostCopy {
    uint32_t dst, src;
};

// A tile is the work of one block: threads (tx, ty, tz) of a TX x TY x TZ
// block (TX = 2^lx, TY = 2^ly, TZ = 2^lz, TX*TY*TZ = kBlock) cover x-index
// x0 + tx, y-index y0 + ty and z-indices z0 + tz + z*TZ for z < zc,
// relative to the box's lower corner; x counts half-row cells (colour
// kernels) or coarse cells (transfer kernels).  Each tile carries its own
// shape, so boxes of different sizes share a launch without idle threads.
struct Tile {
    int box;
    uint16_t x0, y0, z0;
    uint8_t lx, ly, lz, zc;
    uint16_t pad;
};
static_assert(sizeof(Tile) == 16, "tile descriptor size");

struct TileShape {
    int lx, ly, lz;  // log2 of TX, TY, TZ
    int zc;          // z iterations per thread
};

// Face coefficients of a level >= 1: global arrays over the level domain,
// x faces (nx+1)*ny*nz, y faces nx*(ny+1)*nz, z faces nx*ny*(nz+1), F-order.
template <class T>
struct FaceArrays {
    const T* c[3];
    int dlo[3];
    int n[3];  // domain extents
};

// Tiled launch of one level: its boxes, tiles and tile shape.  push != 0:
// every box face is resolvable (RBox::nb), and the kernels that write the
// level's values also write them into the face ghost cells that mirror
// them, so no separate face-ghost refresh is needed.
//
// active != nullptr (batches): a block whose box belongs to a problem slot p
// with active[p] == 0 does nothing.
struct Grid {
    const RBox* boxes;
    const Tile* tiles;
    int ntiles;
    int push;  // producers refresh the face ghosts they mirror; 2: the level is one box
    const int* active;
    int rev;  // walk the tiles in reverse order (see tile_index)
    int res;  // every box's colour blocks span < 2^31 bytes: 32-bit buffer addressing
};

// Transfer launch fine <-> coarse: tiles over the coarse cells of every fine
// box; cbox[b] = coarse box holding the coarsened fine box b.
struct XGrid {
    const RBox* fboxes;
    const RBox* cboxes;
    const int* cbox;
    const Tile* tiles;
    int ntiles;
    int push;  // as Grid::push, for the fine level
    const int* active;
    int rev;
    int res;   // fine and coarse boxes allow 32-bit buffer addressing
};

// One level of the fused coarse V-cycle: a single box in RB storage.
template <class T>
struct CoarseLevel {
    RBox box;  // box.nb[q] == 0: the box itself (periodic), -1: Dirichlet face
    T* u;
    T* f;
    const GhostCopy* face[2];
    long long nface[2];
    const GhostCopy* full;
    long long nfull;
    long long nelem;
    double h;
    FaceArrays<T> fa;  // coefficient faces (c[0] == nullptr: constant coefficient)
    int push;
};

constexpr int kMaxCoarseLevels = 8;

// The levels of the fused coarse cycle, finest first; the last is the bottom.
template <class T>
struct CoarseCycle {
    int nlev;
    int nu1, nu2, prolong;
    int per[3];
    int pid;  // problem slot (checked against the active flags of a batch)
    // lds != 0: u and f of level m live at byte offsets lds_u[m], lds_f[m] of
    // the workgroup's dynamic LDS; the bottom CG's vectors at bot_off
    int lds;
    int lds_u[kMaxCoarseLevels], lds_f[kMaxCoarseLevels];
    int bot_off;
    double rtol;
    int* iters;
    CoarseLevel<T> L[kMaxCoarseLevels];
};

// LDS of the bottom CG over n cells (ngrown with its ghost layer).
inline size_t bottom_lds_bytes(int n, int ngrown) { return 8 * ((size_t)ngrown + 3 * (size_t)n + 40); }
// LDS a workgroup may take on this device (bytes); queried once.
int lds_limit_bytes();

// Per-problem state of a batch, one entry per slot, in device memory.
struct BatchSlot {
    double fnorm;     // max |f| over the valid cells
    double rel_tol, abs_tol;
    int max_cycles;   // ENOCONV past this many cycles
    int fixed_cycles; // > 0: run exactly this many cycles
    int cycles;       // V-cycles done
    int status;       // 0 running / OK, else a bxmg_status
    int nhist;
    int pad;
};
constexpr int kHist = 256;

// ------------------------------------------------------------ launchers
// All launchers enqueue on `s` and return hipSuccess or the launch error.
// active != nullptr: nothing happens while active[0] == 0 (a stopped solve)
hipError_t launch_fill_rb(hipStream_t s, void* data, bool f32, const GhostCopy* list, long long n,
                          const int* active = nullptr);
// hints: NULL, or for every block of kBlock region cells the tag of its
// first cell, then ntags - 1 (tag_hints)
hipError_t launch_fill_fab(hipStream_t s, void* data, bool f32, const FBox* boxes, const Tag* tags, int ntags,
                           long long ncells, int comp0, int ncomp, const int* hints);
// ParallelCopy over region tags (source cell = destination cell + soff)
hipError_t launch_copy_fab(hipStream_t s, bool f32, void* dst, const FBox* dboxes, const void* src,
                           const FBox* sboxes, const Tag* tags, int ntags, long long ncells, int dcomp, int scomp,
                           int ncomp, const int* hints);

// Coefficient modes of the stencil kernels: beta != nullptr -> cell beta of
// the level (same layout as u); fat != nullptr -> face arrays fat[pid] of the
// box's problem; both null -> constant coefficient.  Grid spacing: RBox::h.
// norm_partials != nullptr (FP64, pushing, buffer-addressed levels): also the
// residual norms of the updated cells per tile, as launch_resid writes them.
template <class T>
hipError_t launch_gs(hipStream_t s, const Grid& g, T* u, const T* f, const T* beta, const FaceArrays<T>* fat,
                     int colour, double* norm_partials = nullptr);

// r = f - L u on both colours, optional store of r (R = T, or float for the
// mixed-precision cast), partial norms (max|r|, sum r^2, bad count) at
// 3 * (tile index).  colour0_only (FP64, buffer-addressed, no store): the
// colour-0 cells only, after a colour-1 sweep that took the others' norms.
// nonzero (constant coefficient, buffer-addressed): one flag per problem
// (box pid), set when its guess has a value other than +0.0 or after its
// first check; while it is 0 the residual is f, taken without reading u
// (bitwise the same results as the full path).
template <class T, class R>
hipError_t launch_resid(hipStream_t s, const Grid& g, const T* u, const T* f, const T* beta,
                        const FaceArrays<T>* fat, R* r, double* partials, bool colour0_only = false,
                        const int* nonzero = nullptr);
hipError_t launch_norm_final(hipStream_t s, const double* partials, int n, double* out3);
hipError_t launch_field_norm(hipStream_t s, const Grid& g, const double* x, double* partials);

// uz != nullptr: also zero the coarse u there (its cells and the face ghosts
// that mirror them), in place of zeroing the whole coarse level
template <class T>
hipError_t launch_resid_restrict(hipStream_t s, const XGrid& x, const T* u, const T* f, const T* beta,
                                 const FaceArrays<T>* fat, T* fc, T* uz = nullptr);
template <class T>
hipError_t launch_restrict_plain(hipStream_t s, const XGrid& x, const T* rf, T* fc);
// fine += P coarse: one thread per pair of fine cells (2I, 2I+1) over the
// fine level's colour tiles (fine boxes pair aligned); cbox[b] = coarse box
// holding the coarsened fine box b (plain 32-bit offsets from the box starts:
// buffer addressing measured slower for this kernel).  only_c1: a colour-0
// Gauss-Seidel sweep follows; on levels that push their ghosts, correct the
// colour-1 cells and only the Dirichlet ghosts of colour-0 cells (the sweep
// overwrites colour 0 reading it only through those ghosts).
// stage_values: the largest coarse region (values) a tile of the fine level
// reads (prolong_stage_values); where it fits the LDS stage, the colour-1
// kernel stages it (0: never).  coarse_self: the coarse level is one box, so
// each of its ghosts mirrors one of its own cells (odd reflection across a
// Dirichlet face, the periodic image otherwise); the staged kernel then reads
// those cells instead of the ghosts, which need no refresh before it.
// fine_face_cells > 0: the fine level is one box with that many cells on its
// faces (counted once per face); the staged kernel then leaves the face work
// (ghost pushes, Dirichlet colour-0 ghosts) to a second launch over them.
constexpr int kProlongStage = 2048;  // values of the LDS stage
constexpr long long kSelfGhostCells = 1LL << 18;  // coarse levels up to 64^3 resolve their ghosts in the stage
inline bool prolong_staged(bool fine_push, bool only_c1, int stage_values) {
    return fine_push && only_c1 && stage_values > 0 && stage_values <= kProlongStage;
}
template <class T>
hipError_t launch_prolong(hipStream_t s, const Grid& fine, const RBox* cboxes, const int* cbox, const T* ec, T* uf,
                          int order, bool only_c1 = false, int stage_values = 0, bool coarse_self = false,
                          long long fine_face_cells = 0);

template <class T>
hipError_t launch_zero(hipStream_t s, T* p, long long n, const int* active = nullptr);
hipError_t launch_cast_f32(hipStream_t s, const double* src, float* dst, long long n);

// layout conversions: F-order caller MultiFab (FP64, comp 0) <-> RB level
hipError_t launch_fab_to_rb(hipStream_t s, const Grid& g, const double* fab, const FBox* fb, void* rb, bool f32);
// FP64 launch_fab_to_rb that also sets *nonzero to 1 when any converted value
// is not +0.0 (the caller zeroes it first).
hipError_t launch_fab_to_rb_nz(hipStream_t s, const Grid& g, const double* fab, const FBox* fb, double* rb,
                               int* nonzero);
// launch_fab_to_rb (FP64) and launch_field_norm of the result in one pass
hipError_t launch_fab_to_rb_norm(hipStream_t s, const Grid& g, const double* fab, const FBox* fb, double* rb,
                                double* partials);
// Heat-step right-hand side f = -(u * inv_dt + s) (s == NULL: no source) from
// caller MultiFabs into level storage, with the norms of f per tile.
hipError_t launch_heat_rhs(hipStream_t s, const Grid& g, const double* u, const FBox* fu, const double* src,
                           const FBox* fs, double inv_dt, double* f, double* partials);
hipError_t launch_rb_to_fab(hipStream_t s, const Grid& g, const double* rb, double* fab, const FBox* fb);
hipError_t launch_add_f32(hipStream_t s, const Grid& g, double* u, const float* e);

// periodic projection: subtract the mean of the valid cells
hipError_t launch_mean_sub(hipStream_t s, const Grid& g, double* u, double* scratch);
// Retirement of many problems at once.  Box q of a launch grid belongs to
// problem seg (of the launch) whose tiles are [tstart, tstart + nt) of the
// grid, and writes its solution to fab (FBox f, base relative to fab).
struct RetireBox {
    double* fab;
    FBox f;
    int tstart, nt, seg, pad;
};
// The mean subtraction of launch_mean_sub for every problem of g (bitwise
// the same: each tile's partial sum sits where a launch over that problem
// alone puts it, and each problem's partials are reduced as there);
// seg_tiles[q..q+1] = tile range of problem q (nseg problems); scratch holds
// 3 per tile of g plus 3 per problem.
hipError_t launch_mean_sub_many(hipStream_t s, const Grid& g, const RetireBox* info, const int* seg_tiles, int nseg,
                                double* u, double* scratch);
// launch_rb_to_fab for every box of g into its own problem's MultiFab.
hipError_t launch_rb_to_fab_many(hipStream_t s, const Grid& g, const double* rb, const RetireBox* info);

// variable coefficient setup
template <class T>
hipError_t launch_faces_from_cells(hipStream_t s, const XGrid& x, const T* beta, int d, FaceArrays<T> out, T* dst);
template <class T>
hipError_t launch_faces_coarsen(hipStream_t s, FaceArrays<T> fine, FaceArrays<T> coarse, int d, T* dst);

// bottom: one workgroup, FP64 CG in LDS
template <class T>
hipError_t launch_bottom(hipStream_t s, T* u, const T* f, FaceArrays<T> fa, bool var, const RBox* boxes, int nboxes,
                         const int* dom_lo, const int* dom_hi, const int* periodic, double h, double alpha,
                         double rtol, int* iters_out);

// the fused coarse V-cycle, one workgroup per descriptor cc[0..n); with
// active != nullptr a descriptor whose problem slot is inactive is skipped;
// lds_bytes: dynamic LDS per workgroup (the largest descriptor's need);
// levels_lds: every descriptor has cc.lds set -- the levels then live in
// LDS, otherwise all of them run from device memory (same values either way).
// The cycle zeroes its top level's u itself.
template <class T>
hipError_t launch_coarse_cycle(hipStream_t s, const CoarseCycle<T>* cc, int n, const int* active, bool var,
                               int lds_bytes, bool levels_lds);
// LDS layout of a coarse cycle (sets cc.lds, offsets, bot_off); returns the
// bytes it needs.  Levels go to LDS when everything fits in lds_limit_bytes().
template <class T>
int coarse_lds_layout(CoarseCycle<T>& cc, bool allow_levels);

// ---------------------------------------------------------------- batches
constexpr int kStatusNoConv = -4;     // = BXMG_ENOCONV
constexpr int kStatusNonFinite = -5;  // = BXMG_ENONFINITE

// Per-problem norms: segment q covers partials of tiles [tstart[q],
// tstart[q+1]) and belongs to slot seg_slot[q]; active slots only.
hipError_t launch_norm_seg(hipStream_t s, const double* partials, const int* tstart, const int* seg_slot, int nseg,
                           const int* active, double* norms);
// Stop test of every active member slot (see BatchSlot): records the
// history, retires finished problems, counts the rest into *nactive; seen
// (optional): seen[slot] = 1 for every active slot checked.
hipError_t launch_batch_check(hipStream_t s, const int* slots, int n, const double* norms, BatchSlot* st,
                              int* active, double* hist, double* hist_l2, int* nactive,
                              int* seen = nullptr);
// Ghost lists of many problems in one launch: set q copies list[0..n) with
// indices relative to data + off (active slots only).
struct GhostSet {
    const GhostCopy* list;
    long long n, off;
    int pid, pad;
};
hipError_t launch_fill_sets(hipStream_t s, void* data, bool f32, const GhostSet* sets, int nsets, long long max_n,
                            const int* active);
// Admission of one problem: ||f||_inf from fn3 (max, sum, bad) into st[slot],
// and active[slot] = 1 unless f is zero or not finite.
hipError_t launch_batch_admit(hipStream_t s, const double* fn3, BatchSlot* st, int* active, int slot);
// Admission of n problems in one launch each way: box q of the launch grid g
// reads the caller's initial guess and right-hand side through src[q]
// (pointers, and FBoxes whose bases are relative to them) and writes them
// into level storage u and f through RBox q (bases relative to u and f);
// partials[3 t] receive the right-hand side's norms of tile t (g's tile
// order, so each problem's tiles form one range for launch_norm_seg).
struct ConvSrc {
    const double* phi;
    const double* rhs;
    FBox fphi, frhs;
    int slot;  // the problem's slot: nonzero[slot] |= (its guess has a value other than +0.0)
};
hipError_t launch_admit_convert(hipStream_t s, const Grid& g, const ConvSrc* src, double* u, double* f,
                                double* partials, int* nonzero);
// a[slots[q]] = v for q < n
hipError_t launch_set_slots(hipStream_t s, const int* slots, int n, int* a, int v);
// For q < n: slot = slots[q] takes state states[q] with ||f|| from norms[3 slot]
// and the decision of launch_batch_admit.
hipError_t launch_batch_admit_many(hipStream_t s, const double* norms, const BatchSlot* states, const int* slots,
                                   int n, BatchSlot* st, int* active);
// The same decision with the norms of f reduced from n per-tile partials in
// the same launch (fn3 receives them, as launch_norm_final writes them) and
// the slot state S passed by value instead of copied to st[slot] beforehand.
hipError_t launch_batch_admit_norms(hipStream_t s, const double* partials, int n, const BatchSlot& S, double* fn3,
                                    BatchSlot* st, int* active, int slot);
// Zero element ranges [start, start + len) of the problems still active.
struct ZeroRange {
    long long start, len;
    int pid, pad;
};
template <class T>
hipError_t launch_zero_ranges(hipStream_t s, T* p, const ZeroRange* r, int n, long long max_len, const int* active);

// Scalars of a multigrid-preconditioned conjugate gradient solve, kept on
// the device so that iterations need no host round trip.
struct KrylovScalars {
    double rz;     // r.z of the residual the current direction was built from
    double alpha;  // step along the current direction
    double beta;   // weight of the previous direction in the next one
    double pq;     // p.Lp of the current direction
};
// pn = (double) e + beta p over n elements of a level (ghosts included),
// then e = 0.  e and p must have current face ghosts; pn's follow.
template <class E>
hipError_t launch_kr_axpy(hipStream_t s, E* e, const double* p, double* pn, long long n, const KrylovScalars* sc,
                          const int* active);
// q = L p at every valid cell; partials[3 tile + 1] = the tile's sum of p.q.
hipError_t launch_kr_apply(hipStream_t s, const Grid& g, const double* p, const double* beta, double* q,
                           double* partials);
// x += alpha p, r -= alpha q, rhs = (E) r at every valid cell; partials of
// the new residual's norms as launch_resid writes them.
template <class E>
hipError_t launch_kr_update(hipStream_t s, const Grid& g, double* x, const double* p, double* r, const double* q,
                            E* rhs, const KrylovScalars* sc, double* partials);
// partials[3 tile + 1] = sum of z.q, partials[3 tile + 2] = sum of z.r with
// z = (double) e, over every valid cell.
template <class E>
hipError_t launch_kr_dots(hipStream_t s, const Grid& g, const E* e, const double* r, const double* q,
                          double* partials);
// From reduced sums (sums3[1], sums3[2]): step 0: alpha = rz / (p.q);
// step 1: beta = -alpha (z.q) / rz, then rz = z.r; step 2 (a restart):
// beta = 0, rz = z.r.  Nothing while active[0] == 0.
hipError_t launch_kr_step(hipStream_t s, const double* sums3, KrylovScalars* sc, int step, const int* active);

// Device memory for the allocation-free entry points: a fixed array per GPU
// (kScratchBytes), held until the process ends.  scratch_address() returns
// its address on `device`, which must be the current device; the first call
// per device looks the address up, later calls return the cached value.
constexpr size_t kScratchBytes = size_t(4) << 20;
constexpr int kMaxScratchDevices = 64;
hipError_t scratch_address(int device, void** out);

}  // namespace bxmg
