/*
 * bxmg -- block-structured geometric multigrid for one MI355X (gfx950).
 *
 * C ABI of the library libbxmg.so.  Plain pointers and sizes only; no C++ or
 * PyTorch types cross this boundary, and no exception escapes it.
 *
 * Data model (paper, Section 2): a Box is an inclusive integer index range
 * [lo, hi] (cell centred) in a global index space whose bounds may be
 * negative; a BoxArray is a set of disjoint boxes inside a problem domain; a
 * MultiFab holds, for every box, its data grown by `nghost` ghost cells, in
 * Fortran order (x fastest, then y, z, component), as one device slab.
 * Ghost cells covered by the valid region of some box (after periodic
 * shifts) are filled by FillBoundary, the paper's cached ghost cell exchange
 * (Section 2; fused pack/unpack, Section 3.5).  The multigrid solve is the
 * cell-centred linear solver the paper lists among the framework's functions
 * (Section 2), realised as a red-black Gauss-Seidel V-cycle.
 *
 * Conventions
 *  - Every function returns bxmg_status (0 = BXMG_OK, < 0 = error) unless
 *    stated otherwise; on error bxmg_last_error() gives a message (thread
 *    local, valid until the next failing call of the same thread).
 *  - Handles are owned by the caller and released with the matching
 *    *_release / *_destroy call.  A MultiFab keeps its BoxArray alive.
 *  - Device work is enqueued on the HIP stream passed in (NULL = the
 *    context's stream).  bxmg_mlmg_solve returns after its work completed.
 *  - A caller-provided device buffer stays owned by the caller and must
 *    outlive the MultiFab built on it.
 */
#ifndef BXMG_H
#define BXMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bxmg_ctx_s* bxmg_ctx;
typedef struct bxmg_ba_s* bxmg_boxarray;
typedef struct bxmg_mf_s* bxmg_multifab;

typedef enum {
    BXMG_OK = 0,
    BXMG_EINVAL = -1,     /* invalid argument or geometry                     */
    BXMG_ENOMEM = -2,     /* device or host allocation failed                 */
    BXMG_EDEVICE = -3,    /* a HIP runtime call failed                        */
    BXMG_ENOCONV = -4,    /* max_cycles reached before the tolerance           */
    BXMG_ENONFINITE = -5, /* NaN or Inf seen in the residual or right-hand side */
    BXMG_EBUSY = -6       /* not admitted now (batch memory budget)            */
} bxmg_status;

typedef enum { BXMG_F64 = 0, BXMG_F32 = 1 } bxmg_dtype;
typedef enum { BXMG_PERIODIC = 0, BXMG_DIRICHLET0 = 1 } bxmg_bc;

/* Library version (major*10000 + minor*100 + patch).  Never fails. */
int bxmg_version(void);

/* Message describing the last failure of the calling thread ("" if none). */
const char* bxmg_last_error(void);

/* ------------------------------------------------------------ context ---- */
/* Binds a HIP device and a default stream (NULL = the null stream).  The
 * context owns the multigrid hierarchies it builds (cached per BoxArray and
 * mode) and frees them in bxmg_ctx_destroy, after its stream has drained. */
bxmg_status bxmg_ctx_create(int device, void* hip_stream, bxmg_ctx* out);
void bxmg_ctx_destroy(bxmg_ctx ctx);

/* ----------------------------------------------------------- BoxArray ---- */
/* Host-only calls: no device is needed.
 *
 * bxmg_define_boxarray: chops the domain [dom_lo, dom_hi] (inclusive) into
 * boxes of edge <= max_box_size.  Per direction the blocking factor bf is the
 * largest power of two dividing the domain edge (capped at max_box_size);
 * pieces are floor(max_box_size/bf)*bf long, plus one remainder that is a
 * multiple of bf (e.g. 48 -> 32+16, 240 -> 7x32+16).  bc[d] is a bxmg_bc per
 * direction.  EINVAL for an empty domain or max_box_size < 1. */
bxmg_status bxmg_define_boxarray(const int32_t dom_lo[3], const int32_t dom_hi[3], const int32_t bc[3],
                                 int32_t max_box_size, bxmg_boxarray* out);

/* Explicit box list: lohi is [nboxes][6] = {lo.x, lo.y, lo.z, hi.x, hi.y,
 * hi.z}.  EINVAL if a box is empty, leaves the domain or overlaps another.
 * The boxes need not cover the domain (FillBoundary then leaves the ghosts
 * over the holes untouched); a solve requires full coverage. */
bxmg_status bxmg_define_boxarray_list(const int32_t dom_lo[3], const int32_t dom_hi[3], const int32_t bc[3],
                                      int32_t nboxes, const int32_t* lohi, bxmg_boxarray* out);

/* Number of boxes and (if lohi_out != NULL, room for nboxes*6) their bounds. */
bxmg_status bxmg_boxarray_get(bxmg_boxarray ba, int32_t* nboxes, int32_t* lohi_out);

/* Multigrid level hierarchy the solver builds for this BoxArray: the domain
 * halves while every domain edge is even and >= 4 and every box has an even
 * lower corner and even edges; boxes halve one by one while every box edge is
 * also >= 32, otherwise the coarser level is one box covering its domain.  Writes up to cap_levels
 * levels: lev_nboxes[l], lev_dom[6*l..], and all levels' boxes concatenated
 * in lev_lohi (room for cap_boxes boxes).  EINVAL if a cap is too small. */
bxmg_status bxmg_boxarray_hierarchy(bxmg_boxarray ba, int32_t cap_levels, int32_t* nlevels, int32_t* lev_nboxes,
                                    int32_t* lev_dom, int32_t cap_boxes, int32_t* lev_lohi);
void bxmg_boxarray_release(bxmg_boxarray ba);

/* ----------------------------------------------------------- MultiFab ---- */
/* Bytes of device memory a MultiFab over ba needs: every box's grown data
 * (ncomp * prod(n_d + 2*nghost) elements) starting on a 256-byte boundary. */
size_t bxmg_multifab_bytes(bxmg_boxarray ba, int32_t ncomp, int32_t nghost, bxmg_dtype dtype);

/* Allocates (device_buf == NULL: from the library, freed on release) or
 * adopts (device_buf != NULL: caller-owned device memory of at least
 * bxmg_multifab_bytes bytes, 256-byte aligned) a MultiFab.  Contents are not
 * initialised.  EINVAL for ncomp < 1, nghost < 0 or a misaligned buffer. */
bxmg_status bxmg_alloc_multifab(bxmg_ctx ctx, bxmg_boxarray ba, int32_t ncomp, int32_t nghost, bxmg_dtype dtype,
                                void* device_buf, bxmg_multifab* out);

/* Zero-copy view of box `box` (paper, Section 4.1): device pointer to the
 * first grown cell, grown bounds lo/hi (global indices) and element strides
 * {x, y, z, component}.  EINVAL for a box index out of range. */
bxmg_status bxmg_multifab_box_view(bxmg_multifab mf, int32_t box, void** dptr, int32_t lo[3], int32_t hi[3],
                                   int64_t strides[4]);

/* Slab base pointer and size in bytes, plus ncomp / nghost / dtype. */
bxmg_status bxmg_multifab_info(bxmg_multifab mf, void** base, size_t* bytes, int32_t* ncomp, int32_t* nghost,
                               int32_t* dtype);

/* Copies component `comp` of the valid cells between the MultiFab and a
 * host array over the whole domain in Fortran order (x fastest), of the
 * MultiFab's dtype (to_device != 0: host -> MultiFab).  Ghost cells and the
 * other components keep their values.  Goes through a host copy of the
 * slab; synchronous on hip_stream (NULL = the context's stream). */
bxmg_status bxmg_multifab_copy_host(bxmg_multifab mf, int32_t to_device, void* host, int32_t comp, void* hip_stream);

/* Releases the handle without waiting (paper, Section 3.7: temporaries
 * freed only after the kernels using them finish).  The device memory the
 * library owns for it -- the slab when it allocated one, the box table, the
 * ghost-exchange plans -- is freed in stream order on the context's stream:
 * after the work queued there before the call.  Work that uses the MultiFab
 * on another stream must be ordered before that point by the caller (an
 * event the context's stream waits on) or completed.  A caller-owned slab is
 * left alone. */
void bxmg_multifab_release(bxmg_multifab mf);

/* FillBoundary (paper, Section 2 and Section 3.5): for components
 * [scomp, scomp+ncomp), every ghost cell that -- after wrapping periodic
 * directions -- is a valid cell of some box takes that cell's value; faces,
 * edges and corners (cross == 0) or faces only (cross != 0).  Ghosts outside
 * a non-periodic domain face, and ghosts over uncovered cells, are left
 * untouched.  One fused launch over a cached copy plan.  Asynchronous on
 * `hip_stream`. */
bxmg_status bxmg_fill_boundary(bxmg_multifab mf, int32_t scomp, int32_t ncomp, int32_t cross, void* hip_stream);

/* ParallelCopy (paper, Section 2: copies from one distribution to another):
 * dst and src are MultiFabs over BoxArrays of the same domain and boundary
 * conditions, decomposed differently, of one dtype.  Every cell of a dst box
 * grown by dst_nghost (0 .. dst's nghost) that -- wrapped into the domain
 * through the periodic directions -- lies in the valid region of a src box
 * takes that cell's value, components [scomp, scomp+ncomp) into
 * [dcomp, dcomp+ncomp); other dst cells keep their values.  One fused
 * launch over a region list cached on dst per source BoxArray and width.
 * Asynchronous on hip_stream (NULL = dst's context stream). */
bxmg_status bxmg_parallel_copy(bxmg_multifab dst, int32_t dcomp, bxmg_multifab src, int32_t scomp, int32_t ncomp,
                               int32_t dst_nghost, void* hip_stream);

/* Physical boundary ghosts (homogeneous Dirichlet): every ghost cell outside
 * a non-periodic domain face takes s * (mirror cell), the mirror reflected
 * across every such face (index -1-t -> t below, n+t -> n-1-t above); s = -1
 * per reflected direction when odd != 0, s = +1 otherwise.  Reads the box's
 * own grown data, so call it after bxmg_fill_boundary.  Asynchronous. */
bxmg_status bxmg_apply_domain_bc(bxmg_multifab mf, int32_t scomp, int32_t ncomp, int32_t odd, void* hip_stream);

/* bxmg_fill_boundary for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same result, but the call allocates nothing
 * on the device.  Its copy-region list is built once per MultiFab on the
 * host and staged, on every call, into a fixed per-GPU array of 4 MiB
 * (kept until the process ends) with an asynchronous host-to-device copy on
 * `hip_stream`, which the exchange then reads.  EINVAL when the list needs
 * more than 4 MiB (72 bytes per region: 58254 regions).  Every call on one GPU
 * shares that array: calls on one stream are ordered, calls that overlap on
 * different streams of the same GPU race and must not be issued. */
bxmg_status bxmg_fill_boundary_noalloc(bxmg_multifab mf, int32_t scomp, int32_t ncomp, int32_t cross,
                                       void* hip_stream);

/* -------------------------------------------------------------- solve ---- */
typedef struct {
    int32_t nu1, nu2;       /* pre/post red-black sweeps per level (2, 2)            */
    int32_t max_cycles;     /* cap on V-cycles (200)                                  */
    int32_t precision;      /* 0: FP64 V-cycle; 1: FP32 V-cycle inside FP64 refinement */
    int32_t prolong;        /* 2: trilinear (default); 1: piecewise constant          */
    int32_t fixed_cycles;   /* > 0: run exactly this many cycles, no tolerance stop   */
    double rel_tol;         /* stop when ||f - L u||_inf <= rel_tol * ||f||_inf        */
    double abs_tol;         /*  ... or when ||f - L u||_inf <= abs_tol                 */
    double dx;              /* cell width h (cubic cells); <= 0: 1 / (x-edge of domain) */
    double bottom_rtol;     /* bottom CG relative L2 tolerance (1e-12)                 */
    int32_t krylov;         /* 0: the V-cycles are the iteration; 1: conjugate gradients
                               (flexible form) preconditioned by one V-cycle from zero
                               per iteration, in the precision above (paper Section 2,
                               linear solvers); cycles then counts CG iterations       */
    int32_t reserved;       /* 0                                                      */
    double alpha;           /* >= 0: solve div(beta grad phi) - alpha phi = rhs (Helmholtz;
                               0 = Poisson); with alpha > 0 a fully periodic problem is
                               not singular and no mean is removed                     */
} bxmg_solve_params;

typedef struct {
    int32_t status;         /* bxmg_status of the solve                               */
    int32_t cycles;         /* V-cycles (or refinement steps) performed               */
    int32_t levels;         /* multigrid levels                                       */
    int32_t nhist;          /* entries in hist / hist_l2                              */
    double rel_resid_inf;   /* final ||r||_inf / ||f||_inf                             */
    double resid_l2;        /* final ||r||_2                                          */
    double f_inf;           /* ||f||_inf                                              */
    double seconds;         /* wall time of the solve                                 */
    double hist[256];       /* ||r_k||_inf / ||f||_inf before cycle k                  */
    double hist_l2[256];    /* ||r_k||_2                                              */
} bxmg_solve_info;

/* Fills *p with the defaults above. */
void bxmg_solve_params_default(bxmg_solve_params* p);

/* Solves div(beta grad phi) = rhs on the BoxArray's domain (7-point,
 * cell-centred, h = dx; beta == NULL: beta = 1) with homogeneous Dirichlet
 * (odd-reflection ghosts) or periodic boundaries as the BoxArray's bc says.
 * phi, rhs and beta (if any) must be FP64 MultiFabs over the same BoxArray
 * with nghost >= 1; component 0 is used.  phi's valid cells hold the initial
 * guess on entry (the solver starts from them) and the solution on return;
 * a fully periodic problem returns the mean-zero solution and needs a
 * mean-zero rhs.  The solve is synchronous on the context's stream.
 * Returns info->status: OK, ENOCONV (info filled), ENONFINITE, EINVAL (bad
 * arguments; bottom level above 4096 cells), ENOMEM or EDEVICE. */
bxmg_status bxmg_mlmg_solve(bxmg_ctx ctx, const bxmg_solve_params* params, bxmg_multifab phi, bxmg_multifab rhs,
                            bxmg_multifab beta, bxmg_solve_info* info);

/* One backward-Euler step of the heat equation u_t = div(beta grad u) + s
 * (the heat-equation use of the solvers in the paper's tutorials, Section
 * 4): (u' - u)/dt = div(beta grad u') + s, solved as the Helmholtz problem
 * div(beta grad u') - u'/dt = -(u/dt + s), with the right-hand side formed
 * on the device from u and s and the solve started from u.  u: FP64
 * MultiFab, nghost >= 1, the state on entry and the new state on return
 * (it stays on the device: a time loop calls this once per step).  source:
 * NULL or an FP64 MultiFab over the same boxes (any nghost; valid cells
 * read).  params->alpha is ignored (1/dt is used); the other parameters and
 * the info are those of bxmg_mlmg_solve (rel_tol relative to |f|_inf).
 * EINVAL for dt <= 0 or a non-finite dt. */
bxmg_status bxmg_heat_step(bxmg_ctx ctx, const bxmg_solve_params* params, bxmg_multifab u, bxmg_multifab source,
                           bxmg_multifab beta, double dt, bxmg_solve_info* info);

/* Nodal-centred Poisson solve (the framework's nodal linear solver, paper
 * Section 2): div grad phi = rhs for data at the nodes x = i h, i = 0 .. n_d,
 * of the BoxArray's domain (n_d cells per direction; the solve runs on the
 * whole domain at once, whatever the boxes).  phi and rhs: device arrays of
 * (n_0+1)(n_1+1)(n_2+1) FP64 values, F-order, the domain's lower node first;
 * phi holds the initial guess on entry and the solution on return.  A
 * homogeneous-Dirichlet direction keeps its boundary nodes at 0 (they are
 * not unknowns, rhs is not read there); in a periodic direction node n_d is
 * node 0 (its values are overwritten with node 0's on return), and a fully
 * periodic problem returns the mean-zero solution over the n_0 n_1 n_2
 * distinct nodes.  7-point operator, red-black GS on node parity, full
 * weighting and trilinear transfers, FP64 CG bottom; params as for
 * bxmg_mlmg_solve with precision 0, krylov 0 and alpha 0 only (EINVAL
 * otherwise).  Synchronous. */
bxmg_status bxmg_nodal_solve(bxmg_ctx ctx, const bxmg_solve_params* params, bxmg_boxarray ba, double* phi,
                             const double* rhs, bxmg_solve_info* info);

/* Two-level composite Poisson solve (the block-structured AMR hierarchy of
 * the paper, Sections 1 and 2): div grad phi = rhs on a coarse level over
 * the whole domain and a fine level of refinement ratio 2 over a union of
 * boxes, solved together.  The unknowns are the fine cells and the coarse
 * cells no fine box covers.  Fine ghosts across the coarse-fine boundary are
 * quadratic along the normal through the coarse value and the two fine
 * cells inward, the coarse value being the quadratic (with the mixed term)
 * through the 3x3 coarse cells around the ghost in the face plane; the
 * coarse operator takes the mean of the 4 fine gradients across a face
 * against a covered cell, so the composite operator conserves.  Iteration:
 * fine red-black sweeps, composite residual, one coarse V-cycle from zero,
 * coarse and (trilinear) fine corrections, fine sweeps, covered coarse cells
 * := mean of their children -- repeated until the max composite residual
 * meets rel_tol * max|rhs| (or abs_tol).
 *   phi_c, rhs_c: FP64 MultiFabs over a coarse BoxArray that covers its
 *     domain (any nghost; valid cells used).  On return phi_c holds the
 *     solution at uncovered cells and the mean of the children at covered
 *     ones; rhs_c is read at uncovered cells only.
 *   phi_f, rhs_f: FP64 MultiFabs over the fine BoxArray, whose domain is the
 *     coarse one refined by 2 (lo 2*lo, hi 2*hi+1) with the same boundary
 *     conditions; any nghost (phi_f's valid cells are written, rhs_f's
 *     read, ghost cells left alone; fine boxes that tile one rectangle run
 *     as one merged box in the solver's own storage).  Every
 *     fine box must have even lower and odd upper corners (whole coarse
 *     cells) and lie at least 4 fine cells inside every domain face.
 *   params: nu1, nu2 (fine and coarse sweeps), max_cycles, fixed_cycles,
 *     rel_tol, abs_tol, dx (coarse cell width; <= 0: 1 / coarse x-edge),
 *     bottom_rtol; precision 0, krylov 0, alpha 0, prolong 2 only.
 * Both solutions start from zero (their contents on entry are ignored).
 * Component 0 of each field is used.  A fully periodic problem needs a
 * compatible rhs (zero volume-weighted sum over the unknowns) and returns a
 * solution defined up to a constant.  The per-layout state (one-box coarse
 * fields, the coarse correction's multigrid hierarchy, the fine level's
 * colour-split storage, coverage map, ghost and boundary-cell lists) is
 * cached on the context for the last layout;
 * composite solves on one context run one at a time.
 * Synchronous on the context's stream.  Returns info->status: OK, ENOCONV,
 * ENONFINITE, EINVAL (bad arguments or layout), ENOMEM or EDEVICE. */
bxmg_status bxmg_composite_solve(bxmg_ctx ctx, const bxmg_solve_params* params, bxmg_multifab phi_c,
                                 bxmg_multifab rhs_c, bxmg_multifab phi_f, bxmg_multifab rhs_f,
                                 bxmg_solve_info* info);

/* -------------------------------------------------------------- tuning --- */
/* Launch-shape knobs for hierarchies built after the call (hierarchies are
 * cached per knob setting): param 0 = planes each thread walks in the cell
 * kernels (default 4); param 1 = the same for levels whose tiles span whole
 * box planes (default 4); value in [1, 64].  param 2 = address box data with
 * 32-bit buffer offsets where every box allows it (1, default) or with
 * 64-bit addresses (0).  Other values: EINVAL.  Results do not depend on the
 * knobs; only the work decomposition and instruction selection do.
 * param 3 = at most 2^value threads of a tile along y (0..8, default 8).
 * param 4 = the fused coarse cycle keeps its levels' data in LDS when it
 * fits (1, default) or works on device memory (0).  param 5 = solves run a
 * level whose boxes tile its domain as one box (1, default) or keep the
 * caller's boxes and their ghost exchange on every level (0). */
bxmg_status bxmg_ctx_tune(bxmg_ctx ctx, int32_t param, int32_t value);

/* Launch-shape autotuner: solves the given problem for `cycles` V-cycles
 * (fixed count, params otherwise as given) under every candidate setting of
 * the knobs above -- planes per thread {1, 2, 4, 8} (params 0 and 1), tile
 * rows 2^{2, 3, 8} (param 3), buffer addressing on/off (param 2) -- timing
 * each twice after one warm-up solve, and leaves the fastest set on the
 * context (hierarchies and batches built afterwards use it).  best receives
 * {param 0, param 1, param 2, param 3}, *best_ms the time per V-cycle,
 * *ntried the candidates timed.  phi is overwritten (pass a scratch guess).
 * Synchronous. */
bxmg_status bxmg_autotune(bxmg_ctx ctx, const bxmg_solve_params* params, bxmg_multifab phi, bxmg_multifab rhs,
                          bxmg_multifab beta, int32_t cycles, int32_t best[4], double* best_ms, int32_t* ntried);

/* ---------------------------------------------------------- profiling --- */
/* Kernel timing with HIP events recorded on the context's stream around
 * every launch of one stage on the finest level (level 0) during solves:
 *   0 red-black Gauss-Seidel colour, 1 convergence residual + norms,
 *   2 residual + restriction, 3 prolongation + correction,
 *   4 ghost fills of the solution, 5 the fused coarse cycle (whichever
 *   level it starts at); -1 switches timing off (default).
 * Times accumulate until read; the events add a few microseconds per timed
 * launch to the stream. */
bxmg_status bxmg_profile_stage(bxmg_ctx ctx, int32_t stage);

/* Launches timed and their summed duration in milliseconds since the last
 * reset; reset != 0 clears the totals after reading. */
bxmg_status bxmg_profile_read(bxmg_ctx ctx, int64_t* launches, double* total_ms, int32_t reset);

/* ------------------------------------------------- single level stages --- */
/* The solver's own stage kernels applied once to caller MultiFabs (FP64,
 * nghost >= 1, component 0), each bracketed by the same layout conversion
 * the solver performs on entry and exit.  Synchronous.  h: cell width of
 * the level.  beta may be NULL (constant coefficient).
 *
 * bxmg_gs_colour: ghost exchange + physical ghosts of the other colour, then
 * one red-black colour (colour 0: (i+j+k) even) of Gauss-Seidel,
 * u = (sum_faces beta u_nb - h^2 f) / sum_faces beta, on phi's valid cells. */
bxmg_status bxmg_gs_colour(bxmg_ctx ctx, bxmg_multifab phi, bxmg_multifab rhs, bxmg_multifab beta, double h,
                           int32_t colour);

/* r = rhs - L phi on valid cells (ghost exchange + physical ghosts first);
 * norms[0] = max |r|, norms[1] = sum r^2 (non-finite: norms[0] = NaN). */
bxmg_status bxmg_residual(bxmg_ctx ctx, bxmg_multifab phi, bxmg_multifab rhs, bxmg_multifab beta, double h,
                          bxmg_multifab r, double norms[2]);

/* coarse(I) = (1/8) sum of the 8 children of I; the coarse BoxArray must be
 * the next level of the fine one's hierarchy (or its boxes' coarsening). */
bxmg_status bxmg_restrict(bxmg_ctx ctx, bxmg_multifab fine, bxmg_multifab coarse);

/* fine += P coarse after ghost exchange + physical ghosts of coarse;
 * order 2: trilinear (27/9/3/1 over 64), order 1: piecewise constant. */
bxmg_status bxmg_prolong_add(bxmg_ctx ctx, bxmg_multifab coarse, bxmg_multifab fine, int32_t order);

/* FP64 conjugate-gradient bottom solve on a BoxArray of at most 4096 cells:
 * L phi = rhs from phi = 0, stop at relative L2 residual <= rtol or 4 * cells
 * iterations (fully periodic: rhs projected to mean zero, mean-zero result).
 * *iters receives the iteration count. */
bxmg_status bxmg_bottom_solve(bxmg_ctx ctx, bxmg_multifab phi, bxmg_multifab rhs, bxmg_multifab beta, double h,
                              double rtol, int32_t* iters);

/* ------------------------------------------------------------ batches --- */
/* Many independent problems solved together (the fused multi-box launch of
 * the paper, Section 3.2, taken across problems).  Every stage of the
 * V-cycle is one launch over all boxes of that level of every running
 * problem; the trailing single-box levels of each problem run as one
 * workgroup of one shared launch.  Per cycle: FP64 residual and norms of
 * every problem, a stop test on the device (each problem with its own
 * tolerance), then the V-cycle of those still running; a problem that has
 * stopped costs nothing more.  The cycle is captured as a hipGraph and
 * replayed once the set of running problems has stayed the same for one
 * launch; while problems join or leave every step, its stages are launched
 * one by one instead.
 *
 * Memory: level storage of all problems lives in one arena sized by the
 * budget given at creation (the arena is the budget; nothing else grows
 * with the number of problems except small per-problem tables).  A problem
 * is admitted only if its levels fit in the free part of the arena (the
 * admission by HBM footprint the serving loop needs); problems keep their
 * storage on the device until they finish.
 *
 * Every problem's result is the one bxmg_mlmg_solve gives for it alone with
 * the batch's parameters: the same kernels in the same order per problem,
 * and stop tests on exact max-norms.  */
typedef struct bxmg_batch_s* bxmg_batch;

/* params: shared by all problems (NULL = defaults; precision 1 = FP32
 * V-cycle inside FP64 refinement); var != 0: every problem brings a beta
 * MultiFab, var == 0: none does.  max_problems: slots (1..4096).
 * hbm_budget_bytes: arena plus coefficient storage (at most 2^31 elements
 * per arena array).  Each call takes the context's lock. */
bxmg_status bxmg_batch_create(bxmg_ctx ctx, size_t hbm_budget_bytes, int32_t max_problems, int32_t var,
                              const bxmg_solve_params* params, bxmg_batch* out);
void bxmg_batch_destroy(bxmg_batch b);

/* Device bytes problem `ba` would take in batch b (0 if it cannot run in a
 * batch: a domain whose trailing levels are not single boxes of at most 4096
 * cells, or level storage beyond 2^31 elements). */
size_t bxmg_batch_footprint(bxmg_batch b, bxmg_boxarray ba);

/* Admits a problem: takes its slot and arena range now; the conversion of
 * phi (initial guess), rhs (and beta) into the arena and ||rhs||_inf run at
 * the next bxmg_batch_step / bxmg_batch_launch, together with every problem
 * added since the last one, after the work the caller queued on the
 * context's stream before that call (phi, rhs and beta must keep their
 * values until then; a zero or non-finite rhs retires the problem at that
 * step).  rel_tol <= 0: the batch's rel_tol.  The MultiFabs (FP64, nghost >= 1,
 * one BoxArray) must stay alive until the result is polled: phi receives
 * the solution.  BXMG_EBUSY: the footprint does not fit now or every slot
 * is taken (nothing changed); EINVAL: bad arguments or a domain a batch
 * cannot run.  *id identifies the problem in poll / remove. */
bxmg_status bxmg_batch_add(bxmg_batch b, bxmg_multifab phi, bxmg_multifab rhs, bxmg_multifab beta, double rel_tol,
                           int64_t* id);

/* Runs ncycles (>= 1) batch cycles, then synchronises once, writes the
 * solutions of the problems that stopped into their phi and queues their
 * results for poll.  *nrunning (may be NULL): problems still running. */
bxmg_status bxmg_batch_step(bxmg_batch b, int32_t ncycles, int32_t* nrunning);

/* bxmg_batch_step in two halves, so that the cycles of several batches
 * (each on its own stream) overlap on the device: launch enqueues ncycles
 * cycles and returns at once (EBUSY if an earlier launch is not collected);
 * collect waits for them and does the rest of a step.  add, remove and set
 * are refused (EINVAL) between the two. */
bxmg_status bxmg_batch_launch(bxmg_batch b, int32_t ncycles);
bxmg_status bxmg_batch_collect(bxmg_batch b, int32_t* nrunning);

/* Up to max finished problems, oldest first: ids[i] and infos[i] (status,
 * cycles, history; seconds = time from add to the end of its last step).
 * *ndone receives the number returned. */
bxmg_status bxmg_batch_poll(bxmg_batch b, int32_t max, int64_t* ids, bxmg_solve_info* infos, int32_t* ndone);

/* Cancels a running problem (its phi keeps whatever it held) or drops a
 * finished one from the poll queue.  EINVAL for an unknown id. */
bxmg_status bxmg_batch_remove(bxmg_batch b, int64_t id);

/* Occupancy: device bytes in use by problems, the budget, running problems,
 * finished problems waiting in the poll queue (any pointer may be NULL). */
bxmg_status bxmg_batch_stats(bxmg_batch b, size_t* bytes_used, size_t* bytes_budget, int32_t* nrunning,
                             int32_t* nqueued);

/* Knobs: param 0 = capture the cycle as a hipGraph (value 1, default) or
 * launch it stage by stage (0).  Results do not depend on it. */
bxmg_status bxmg_batch_set(bxmg_batch b, int32_t param, int32_t value);

#ifdef __cplusplus
}
#endif
#endif /* BXMG_H */
