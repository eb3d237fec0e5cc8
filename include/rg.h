/*
 * rg.h -- C ABI of the MI355X (gfx950) library for the per-level
 * hydrodynamics update on a cell-by-cell oct tree, after RAMSES-GPU
 * (Teyssier et al., arXiv 2607.20704).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers named d_* are device memory owned by the caller; pointers named
 *   h_* are host memory read (or written) during the call only.  The library
 *   allocates no device memory in any call below except rg_sort_keys'
 *   caller-sized workspace use and rg_batch_create (which owns only its
 *   graph and a small device table, released by rg_batch_destroy).
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *   work is enqueued asynchronously on it; nothing synchronises unless the
 *   description says so.
 * - Every call returns an rg_status.  Calls never abort, throw or print.  On
 *   an argument error nothing is enqueued and the outputs are untouched.
 *   rg_last_error_detail() returns a thread-local text for the last failure.
 * - Errors found on the device (duplicate key, ungraded tree, full table,
 *   non-finite state, a flux owed to a coarse cell with no buffer) are
 *   recorded in the hash workspace header of the tree the call works on
 *   (rg_step, rg_step_subcycled, rg_batch_*; rg_hash_build and the
 *   neighbour build) and reported by rg_check(d_ws).  Calls given no
 *   workspace (rg_hydro_step_level, rg_cfl_dt, rg_cfl_dt_corrected outside
 *   a step) record them in the library's own error word on the current
 *   device, reported and cleared by rg_check(NULL).
 * - Non-finite states: every CFL reduction also watches the cells it reads
 *   for a NaN or infinite density, energy or signal speed |u|+|v|+|w|+3c.
 *   On one it writes the time step 0 -- no finite state gives 0 and no later
 *   limit can raise it, so later updates change no finite cell -- and
 *   records RG_ENONFINITE.
 * - Results are deterministic: identical inputs give identical bits.  There
 *   are no floating-point atomics on the update path.
 *
 * Tree and state layout
 * ---------------------
 * - Level l (1 <= l <= RG_MAX_LEVEL) of the unit box has 2^l cells and
 *   2^(l-1) octs per side; an oct is the 2x2x2 cell block (i,j,k,l) (Sec. 2).
 * - Octs are stored in ascending key order: by level, then along a 3-D
 *   Hilbert curve (Sec. 2.2 and Fig. 1).  Key of oct (i,j,k,l):
 *       K = 2^(3(l-1)) + H_(l-1)(i,j,k)
 *   where H_b is Skilling's Hilbert index (AIP Conf. Proc. 707, 2004)
 *   evaluated at order 20 on (i,j,k) * 2^(20-b) and shifted right by
 *   3(20-b).  The parent key is K >> 3; no key is zero.
 * - Cell c of oct o has global id 8*o + c, c = ix + 2*iy + 4*iz.
 * - State: double U[8*n_oct][5], variables (rho, rho*u, rho*v, rho*w, E),
 *   ideal gas.  Floors rho >= RG_RHO_MIN and p >= RG_P_MIN are applied to
 *   primitive variables.
 * - Neighbour list (Sec. 2.1, 2.3; the 27-entry list of Sec. 5):
 *   int32 nbr27[n_oct][27], entry (dx+1) + 3(dy+1) + 9(dz+1) for the oct
 *   offset (dx,dy,dz) in {-1,0,1}^3 (entry 13 is the oct itself):
 *       e >= 0         same-level oct index
 *       e <= -1        the missing oct is covered by coarse leaf cell -1-e
 *       RG_NBR_OUTSIDE outside the domain (outflow boundaries)
 * - father_cell[o]: global id of the level-(l-1) cell that oct o refines,
 *   -1 on the coarsest level.  son_mask[o]: bit c set iff cell c of oct o has
 *   a child oct (32-bit word per oct, low 8 bits used).
 * - Empty inputs: a call given a zero count or an empty oct range does
 *   nothing and returns RG_OK, and its device pointers may then be null.
 *   Exceptions: rg_hash_build with n = 0 still writes an empty table (its
 *   workspace must be valid; every lookup then returns -1), rg_level_ranges
 *   with n = 0 writes zeros, and rg_cfl_dt over levels that hold no octs
 *   writes +inf (its pointers must still be valid).
 */
#ifndef RG_H
#define RG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RG_ABI_VERSION 13
#define RG_MAX_LEVEL 21
#define RG_NBR_OUTSIDE INT32_MIN
#define RG_RHO_MIN 1e-10
#define RG_P_MIN 1e-20

typedef enum rg_status {
    RG_OK = 0,
    RG_EINVAL = 1,       /* bad argument: null/misaligned pointer, size, level, enum */
    RG_EFULL = 2,        /* hash workspace too small for the keys */
    RG_EDUPKEY = 3,      /* a key was inserted twice */
    RG_EUNGRADED = 4,    /* a missing neighbour has no coarse cell under it */
    RG_ENONFINITE = 5,   /* a NaN or infinite state met by a time-step reduction */
    RG_EHIP = 6,         /* a HIP runtime call failed (text in the detail) */
    RG_ENOTSUP = 7       /* unsupported device or configuration */
} rg_status;

enum { RG_BC_PERIODIC = 0, RG_BC_OUTFLOW = 1 };

/* Coarse ghost cells (Sec. 2.3: ghost zones where a neighbour oct is
 * missing; the paper does not say how they are filled).  INJECT: every fine
 * position takes the coarse cell's values.  LINEAR: minmod-limited linear
 * interpolation of the conserved variables inside the coarse cell C: slope_a
 * = minmod(U_C - U_a-, U_a+ - U_C) from C's face neighbours (same-level
 * cells, else the coarser cell covering them, C itself across an outflow
 * face), and a fine cell at sub-position s gets ((U_C + q_x slope_x) + q_y
 * slope_y) + q_z slope_z, q = -1/4 for s = 0 and +1/4 for s = 1.  Selected
 * per tree (rg_tree.ghost); rg_hydro_step_level, which has no tree, injects. */
enum { RG_GHOST_INJECT = 0, RG_GHOST_LINEAR = 1 };

/* Precision forms of the hydro update:
 *   RG_FP64  every step in double precision.
 *   RG_MIXED primitive variables (including pressure) computed in double
 *            from the double state, then rounded to float; slopes,
 *            predictor, face states and HLLC in float; each face flux is
 *            widened to double, scaled by dt/dx and accumulated in double,
 *            the same value entering both neighbours (so mass, momentum and
 *            energy are conserved to double rounding).  dt stays double. */
enum { RG_FP64 = 0, RG_MIXED = 1 };

const char *rg_status_string(int status);

/* Copies the thread-local detail of the last failed call (NUL-terminated,
 * truncated to len) and returns its full length. */
size_t rg_last_error_detail(char *buf, size_t len);

/* Library ABI version (RG_ABI_VERSION). */
int rg_abi_version(void);

/* ---------------------------------------------------------------------- */
/* Keys and order (Sec. 2.1 key tuple; Sec. 2.2 level sort + Hilbert sort) */
/* ---------------------------------------------------------------------- */

/* Keys of n octs: d_ijkl is int32[n][4] = (i, j, k, l) with 1 <= l <= 21 and
 * 0 <= i,j,k < 2^(l-1); d_keys is uint64[n].  Out-of-range input gives key 0,
 * which rg_hash_build rejects (RG_EINVAL via rg_check). */
rg_status rg_encode_keys(const int32_t *d_ijkl, int64_t n, uint64_t *d_keys, void *stream);

/* Host evaluation of the same key function the kernels use (testing aid):
 * returns K for (i,j,k,l), 0 if out of range. */
uint64_t rg_key_host(int32_t i, int32_t j, int32_t k, int32_t l);

/* Host inverse of rg_key_host for a valid key: writes (i,j,k,l) to h_ijkl[4]. */
void rg_key_coords_host(uint64_t key, int32_t *h_ijkl);

/* Inverse of rg_encode_keys: d_ijkl[n][4] from valid keys. */
rg_status rg_decode_keys(const uint64_t *d_keys, int64_t n, int32_t *d_ijkl, void *stream);

/* Device workspace needed by rg_sort_keys for n keys. */
size_t rg_sort_workspace_bytes(int64_t n);

/* Sorts n keys ascending (LSD radix sort over the 64-bit keys) into
 * d_keys_out and writes d_perm[r] = input position of the r-th key
 * (int32).  d_ws must hold rg_sort_workspace_bytes(n) bytes. */
rg_status rg_sort_keys(const uint64_t *d_keys_in, int64_t n, uint64_t *d_keys_out, int32_t *d_perm,
                       void *d_ws, size_t ws_bytes, void *stream);

/* First oct of every level in sorted keys: d_level_begin is
 * int64[RG_MAX_LEVEL + 2]; octs of level l are [begin[l], begin[l+1]). */
rg_status rg_level_ranges(const uint64_t *d_sorted_keys, int64_t n, int64_t *d_level_begin, void *stream);

/* Gathers per-oct rows: d_out[r] = d_in[d_perm[r]] for rows of `row_doubles`
 * doubles (40 for a cell state of one oct).  Used to put the state in key
 * order. */
rg_status rg_permute_rows(const double *d_in, const int32_t *d_perm, int64_t n_rows, int row_doubles,
                          double *d_out, void *stream);

/* ---------------------------------------------------------------------- */
/* Hash table (Sec. 2.1: fnv64 hash with linear probing; Sec. 6: CAS insert) */
/* ---------------------------------------------------------------------- */

/* Workspace for n keys: a 256-byte header, then capacity = the power of two
 * >= 2n (load factor <= 1/2) slots of uint64 keys and int32 values, then the
 * scratch of the build (about 17 n bytes). */
size_t rg_hash_workspace_bytes(int64_t n_keys);

/* Clears the table and inserts (d_keys[i], i) for i < n: slot = FNV-1a-64
 * over the 8 little-endian key bytes, masked by capacity - 1, then linear
 * probing.  Built segment by segment: keys are bucketed by the 4096-slot
 * segment of their home slot (a counting sort: per-chunk counts, their
 * prefix, a scatter), each segment is filled in LDS with 64-bit
 * compare-and-swap and written out whole, and the few probe sequences that
 * leave their segment are finished with global compare-and-swap.  Keys must
 * be non-zero and unique; violations are flagged in the header (rg_check).
 * Slot positions depend on insertion order; only lookups are defined. */
rg_status rg_hash_build(const uint64_t *d_keys, int64_t n, void *d_ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * build as rg_hash_build, same table, same lookups, with the build's scratch
 * taken from a static device array of the library instead of the caller's
 * workspace.  d_table (256-byte aligned, caller-owned) receives only the
 * table: the 256-byte header and the slots, at least
 * ((256 + capacity * 12 + 255) / 256) * 256 bytes, capacity being the power of
 * two >= max(2n, 16); a buffer of rg_hash_workspace_bytes(n) bytes also
 * fits.  The result is read by rg_hash_lookup, rg_check and
 * rg_build_neighbours like a workspace rg_hash_build filled.
 * Limits: n <= 4,194,304 keys (RG_EINVAL above, before any launch); a table
 * smaller than the above is RG_EFULL.  The static array (about 72 MiB) is
 * held by every device that runs this call, from its first call until the
 * process ends.  Calls allocate nothing (no hipMalloc, hipFree or allocating
 * library routine) and need no clearing between them: every call writes each
 * scratch word before it reads it.  All calls on one device share that
 * device's array: calls that overlap in time on one device (on different
 * streams, or from different threads) race and give undefined tables. */
rg_status rg_hash_build_noalloc(const uint64_t *d_keys, int64_t n, void *d_table, size_t table_bytes, void *stream);

/* The paper's hash_get: d_idx[i] = index of key d_q[i], or -1 if absent. */
rg_status rg_hash_lookup(const void *d_ws, const uint64_t *d_q, int64_t m, int32_t *d_idx, void *stream);

/* Synchronises `stream` and returns the first device-side error recorded in
 * the workspace since the last rg_hash_build (RG_OK if none); *h_bad_index
 * receives the offending key or oct index (or -1).  With d_ws NULL it
 * returns, and clears, the library's own error word of the current device
 * (errors of calls that were given no workspace). */
rg_status rg_check(const void *d_ws, int64_t *h_bad_index, void *stream);

/* FNV-1a-64 of the 8 little-endian bytes of `key`, computed on the host with
 * the same code the kernels use (offered for testing against the published
 * FNV definition). */
uint64_t rg_fnv1a64(uint64_t key);

/* ---------------------------------------------------------------------- */
/* Neighbour lists (Sec. 2.1 hash_get; Sec. 2.3 ghost zones; Sec. 5 nbor)   */
/* ---------------------------------------------------------------------- */

/* For n key-ordered octs whose keys are in the hash table d_ws: writes
 * nbr27[n][27], father_cell[n] and son_mask[n] (layout above).  Each oct's
 * coordinates come from decoding its key; each neighbour is found by
 * encoding its key and probing the table, then, if absent, probing its
 * father key (K >> 3) for the coarse cell underneath.  `lmin` is the
 * coarsest level present.  A missing neighbour without coarse cell, or an
 * oct above lmin without father, sets RG_EUNGRADED in the workspace
 * (rg_check).  bc is RG_BC_PERIODIC or RG_BC_OUTFLOW. */
rg_status rg_build_neighbours(void *d_ws, const uint64_t *d_keys, int64_t n, int lmin, int bc,
                              int32_t *d_nbr27, int32_t *d_father_cell, uint32_t *d_son_mask, void *stream);

/* ---------------------------------------------------------------------- */
/* Hydro update (Sec. 3: MUSCL-Hancock + HLLC, uold -> unew)              */
/* ---------------------------------------------------------------------- */

/* Kernel choice; zero-initialised means "library default". */
typedef struct rg_tuning {
    int32_t octs_per_group;   /* per-oct kernel: octs handled by one workgroup (0 = default) */
    int32_t threads;          /* per-oct kernel: workgroup size (0 = default) */
    int32_t no_bricks;        /* 1: scheduled updates use the per-oct kernel for every oct */
    int32_t persistent;       /* batched form: 1 = persistent grids looping over the work list,
                                 0 = one workgroup per work item */
    int32_t brick_waves;      /* brick kernel register budget: waves per SIMD it is compiled for
                                 (FP64: 2 or 3, mixed: 3 or 4; 0 = default: 2 for FP64, 3 mixed) */
    int32_t no_groups;        /* 1: scheduled updates leave complete sibling groups to the per-oct kernel */
    int32_t group_threads;    /* sibling-group kernel workgroup size: 256, 320 or 384 (0 = default) */
    int32_t no_pairs;         /* 1: a complete periodic finest level's bricks one by one, not two
                                 stacked along z per workgroup (the same bits either way) */
} rg_tuning;

/* Kernel schedule of a tree.  A brick is a Hilbert-aligned cube of 8x8x8
 * octs of one level (keys 512 P .. 512 P + 511, so consecutive in memory);
 * a complete brick none of whose octs borders a coarse ghost is updated by
 * the brick kernel, which marches the brick plane by plane and shares the
 * stencil of all its octs (the paper's larger-block idea, Sec. 3); all other
 * octs are updated one at a time, or eight at a time where they form a
 * complete sibling group (the 8 children of one oct, keys 8 P .. 8 P + 7,
 * consecutive in memory), whose 4^3 cells share one stencil tile.  For level
 * l, d_list holds [brick_begin[l], +brick_count[l]) first octs of bricks,
 * [rest_begin[l], +rest_count[l]) every oct outside them, and that set split
 * into [group_begin[l], +group_count[l]) first octs of complete sibling
 * groups (levels above lmin) and [single_begin[l], +single_count[l]) the
 * other octs.  The schedule depends only on the keys and neighbour lists:
 * rebuild it when the tree changes. */
typedef struct rg_schedule {
    int64_t brick_begin[RG_MAX_LEVEL + 2];
    int64_t brick_count[RG_MAX_LEVEL + 2];
    int64_t rest_begin[RG_MAX_LEVEL + 2];
    int64_t rest_count[RG_MAX_LEVEL + 2];
    /* neighbour-list build: every complete brick (coarse neighbours allowed;
     * only the slots around the brick are hashed) and the other octs */
    int64_t nbr_brick_begin, nbr_brick_count;
    int64_t nbr_rest_begin, nbr_rest_count;
    /* coarse-fine corrections: the octs of level l (> lmin) with a coarse
     * cell across one of their six faces */
    int64_t border_begin[RG_MAX_LEVEL + 2];
    int64_t border_count[RG_MAX_LEVEL + 2];
    int64_t group_begin[RG_MAX_LEVEL + 2];
    int64_t group_count[RG_MAX_LEVEL + 2];
    int64_t single_begin[RG_MAX_LEVEL + 2];
    int64_t single_count[RG_MAX_LEVEL + 2];
    const int32_t *d_list;
} rg_schedule;

/* Bytes of the coarse-fine correction buffer for octs [corr_base, n_oct):
 * 30 doubles (6 sides x 5 variables) per oct. */
size_t rg_corr_workspace_bytes(int64_t n_octs);

/* One level's update (Sec. 3): for the octs [oct_begin, oct_end) of one
 * level, with cell size dx and the time step *d_dt (device scalar):
 *   - gathers the 6x6x6 stencil of each oct: same-level neighbours give
 *     their cells, a missing neighbour gives its coarse cell to all 8
 *     positions (injection), outside positions copy the nearest cell in the
 *     domain (zero gradient);
 *   - primitive variables, minmod slopes of primitives along x, y, z, the
 *     Hancock half step W' = W - dt/(2dx) sum_d A_d(W) dW_d, face states
 *     W' -/+ dW_d/2 (floored);
 *   - HLLC flux (Davis speeds, side-symmetric star state) on the 36 faces of
 *     the oct's cells, G = F dt/dx, set to zero on a face touching a split
 *     cell;
 *   - unew = ((uold + (Gx- - Gx+)) + (Gy- - Gy+)) + (Gz- - Gz+) for the
 *     oct's 8 cells;
 *   - for each side bordering a coarse cell, writes the flux owed to it,
 *     +/- (1/8) ((G00 + G10) + (G01 + G11)), into
 *     d_corr[30 * (o - corr_base) + 5 * side + var] (side = 2 * axis +
 *     high); d_corr may be NULL only if no oct in the range has a coarse
 *     neighbour: an oct that has one is reported as RG_EINVAL (index: the
 *     oct) in the error word (rg_check(NULL), or the tree's workspace
 *     inside rg_step), its owed fluxes being lost;
 *   - if d_dt_next is not NULL (device double, set to +inf by the caller
 *     before the first level of a step), folds into it with a 64-bit
 *     atomicMin the CFL limit cfl dx / (|u|+|v|+|w|+3c) of the new state of
 *     every leaf cell of the range that has no split face neighbour (the
 *     cells the coarse-fine correction leaves alone; rg_cfl_dt_corrected
 *     covers the others).  Together they give, bit for bit, what rg_cfl_dt
 *     returns on the finished new state, without another pass over it.
 * uold and unew must not overlap.  form is RG_FP64 or RG_MIXED; tune may be
 * NULL. */
rg_status rg_hydro_step_level(double dx, const double *d_dt, double gamma,
                              const double *d_uold, double *d_unew,
                              const int32_t *d_nbr27, const uint32_t *d_son_mask,
                              int64_t oct_begin, int64_t oct_end,
                              double *d_corr, int64_t corr_base,
                              double cfl, double *d_dt_next,
                              int form, const rg_tuning *tune, void *stream);

/* Adds the fluxes recorded by rg_hydro_step_level for octs [oct_begin,
 * oct_end) to the coarse cells they border: for side = 0..5 in turn, every
 * oct whose neighbour across that side is coarse cell C does
 * unew[C] += d_corr[30 * (o - corr_base) + 5 * side + v].  One launch per
 * side; within a side no two octs share a target, so no atomics are used. */
rg_status rg_apply_coarse_corrections(double *d_unew, const double *d_corr, int64_t corr_base,
                                      const int32_t *d_nbr27, int64_t oct_begin, int64_t oct_end, void *stream);

/* Upload (Table 1 "hydro - upload"): for octs [oct_begin, oct_end) of one
 * level, u[father_cell[o]] = 0.125 * (((c0+c1)+(c2+c3))+((c4+c5)+(c6+c7))).
 * Octs without a father cell (father_cell -1: the coarsest level) are
 * skipped. */
rg_status rg_restrict_level(double *d_u, const int32_t *d_father_cell, int64_t oct_begin, int64_t oct_end,
                            void *stream);

/* CFL time step (Table 1 "compute dt"): *d_dt = cfl * min over leaf cells of
 * dx_l / (|u| + |v| + |w| + 3 c), c = sqrt(gamma p / rho), dx_l = 2^-l.
 * h_level_begin[l] (host, int64[RG_MAX_LEVEL + 2]) gives the level ranges;
 * the minimum is taken with a 64-bit atomicMin on the bits of positive
 * doubles, so the result is exact and order independent. */
rg_status rg_cfl_dt(const double *d_u, const uint32_t *d_son_mask, const int64_t *h_level_begin,
                    int lmin, int lmax, double gamma, double cfl, double *d_dt, void *stream);

/* Folds into *d_dt (atomicMin, no reset) the CFL limit of every coarse cell
 * that borders an oct above lmin across a face -- the cells that
 * rg_apply_coarse_corrections changes -- from d_u (call it after the
 * corrections).  With the d_dt_next output of the level updates this
 * completes the next step's time step. */
rg_status rg_cfl_dt_corrected(const double *d_u, const int32_t *d_nbr27, const int64_t *h_level_begin, int lmin,
                              int lmax, double gamma, double cfl, double *d_dt, void *stream);

/* ---------------------------------------------------------------------- */
/* Whole step on one tree                                                 */
/* ---------------------------------------------------------------------- */

typedef struct rg_tree {
    int64_t n_oct;
    int32_t lmin, lmax;                       /* levels present */
    int32_t bc;                               /* RG_BC_* */
    int32_t ghost;                            /* coarse ghost cells: RG_GHOST_INJECT or RG_GHOST_LINEAR */
    int64_t level_begin[RG_MAX_LEVEL + 2];    /* host copy of the level ranges */
    uint64_t *d_keys;                         /* sorted keys [n_oct] */
    void *d_hash_ws;                          /* rg_hash_workspace_bytes(n_oct) */
    size_t hash_ws_bytes;
    int32_t *d_nbr27;                         /* [n_oct][27] */
    int32_t *d_father_cell;                   /* [n_oct] */
    uint32_t *d_son_mask;                     /* [n_oct] */
    double *d_corr;                           /* 30 doubles per oct of levels > lmin; NULL if lmin == lmax */
    /* used by RG_STEP_REKEY only (may be NULL otherwise): */
    int32_t *d_ijkl;                          /* key-ordered oct coordinates [n_oct][4] */
    uint64_t *d_keys_scratch;                 /* [n_oct] unsorted keys */
    int32_t *d_perm;                          /* [n_oct] sort permutation (identity for a static tree) */
    void *d_sort_ws;                          /* rg_sort_workspace_bytes(n_oct) */
    size_t sort_ws_bytes;
    int64_t *d_level_begin;                   /* device level ranges [RG_MAX_LEVEL + 2] */
    const rg_schedule *sched;                 /* optional kernel schedule (NULL: per-oct kernel) */
    int64_t capacity;                         /* octs every per-oct buffer can hold (ngridmax, Sec. 2);
                                                 0: n_oct.  rg_refine may grow the tree up to it. */
} rg_tree;

/* Builds the schedule of tree t (keys, level ranges and neighbour lists must
 * be current) into the caller's d_list (capacity >= 4 n_oct int32 entries).
 * Reads the keys and neighbour lists back to the host: synchronises.  Once
 * t->sched points to it, rg_prepare_tree builds neighbour lists brick by
 * brick. */
rg_status rg_schedule_build(const rg_tree *t, int32_t *d_list, int64_t capacity, rg_schedule *out, void *stream);

/* Bytes of the workspace rg_schedule_build_device needs for n_oct octs. */
size_t rg_schedule_workspace_bytes(int64_t n_oct);

/* The same schedule built on the device (no copy of the tree to the host;
 * synchronises once to read the list lengths back): per level the same
 * brick, per-oct, border, sibling-group and single-oct lists, in key order,
 * list by list (offsets in *out).  d_list capacity >= 4 n_oct; d_ws is
 * rg_schedule_workspace_bytes(n_oct) bytes, 256-byte aligned.  For trees
 * that change every step (rg_refine). */
rg_status rg_schedule_build_device(const rg_tree *t, int32_t *d_list, int64_t capacity, void *d_ws, size_t ws_bytes,
                                   rg_schedule *out, void *stream);

/* One level's update following a schedule: the level's bricks with the
 * brick kernel, its complete sibling groups with the sibling-group kernel
 * (one 8x8x8 tile per group; tune->no_groups 1 leaves them to the per-oct
 * kernel), its other octs with the per-oct kernel (the last two also record
 * the coarse-side fluxes in t->d_corr).  Same results, bit for bit, as
 * rg_hydro_step_level over the whole level. */
rg_status rg_hydro_step_scheduled(const rg_tree *t, const rg_schedule *sched, int level, const double *d_dt,
                                  double gamma, const double *d_uold, double *d_unew, double cfl, double *d_dt_next,
                                  int form, const rg_tuning *tune, void *stream);

#define RG_STEP_REBUILD 1u    /* rebuild the hash table and neighbour lists first */
#define RG_STEP_REKEY 2u      /* recompute keys from d_ijkl, radix-sort them, level ranges */
#define RG_STEP_CHAIN_DT 4u   /* d_dt[0] holds this step's dt; the next step's goes to d_dt[1] */

/* The tree bookkeeping of a step (Sec. 2.1-2.3; Table 1 "refine"/"cache"
 * rows for a static tree): with RG_STEP_REKEY, keys from d_ijkl, radix sort
 * into d_keys / d_perm and device level ranges; with RG_STEP_REBUILD, hash
 * build from d_keys and neighbour lists.  Errors found on the device are
 * reported by rg_check(d_hash_ws). */
rg_status rg_prepare_tree(const rg_tree *t, unsigned flags, void *stream);

/* One step with a global time step (no subcycling):
 *   rg_prepare_tree(t, flags & (REBUILD | REKEY)) (nothing when none is set);
 *   dt = rg_cfl_dt(uold) into *d_dt -- or, with RG_STEP_CHAIN_DT, d_dt[0]
 *   is taken as this step's dt (from the previous chained step or from
 *   rg_cfl_dt) and the next step's dt is computed from unew inside the level
 *   updates plus rg_cfl_dt_corrected into d_dt[1], saving the separate pass
 *   over the state (so a chain of steps s = 0, 1, ... passes d_dt + s);
 *   every level: rg_hydro_step_scheduled if t->sched is set, else
 *   rg_hydro_step_level over the level (uold -> unew);
 *   rg_apply_coarse_corrections over all levels above lmin (restricted to
 *   the schedule's border lists when t->sched is set: same bits);
 *   rg_restrict_level from lmax down to lmin + 1 on unew.
 * The caller swaps uold and unew afterwards. */
rg_status rg_step(const rg_tree *t, const double *d_uold, double *d_unew, double gamma, double cfl, int form,
                  unsigned flags, double *d_dt, const rg_tuning *tune, void *stream);

/* One coarse step with level subcycling (Sec. 2: adaptive time steps level
 * by level, each level taking two steps of half its parent's):
 *   rg_prepare_tree(t, flags) (flags: RG_STEP_REBUILD, RG_STEP_REKEY or 0);
 *   d_dt[0] = D = cfl * min over leaf cells of 2^(l - lmin) dx_l /
 *   (|u|+|v|+|w|+3c), the coarse step; d_dt[1 + k] = D / 2^k, the step of
 *   level lmin + k (d_dt: device, double[2 + lmax - lmin]);
 *   advance(lmin, D), where advance(l, dt) is: level l's update with dt (as
 *   rg_hydro_step_level; its coarse ghost cells take the coarser level's
 *   values from the start of that level's current step); if l < lmax, twice
 *   { advance(l + 1, dt / 2) }, with acc = (0 + first substep's coarse-side
 *   fluxes of level l+1) + second substep's,
 *   then acc added to the coarse cells side by side (as
 *   rg_apply_coarse_corrections) and level l+1 restricted into level l.
 * The fine fluxes of both substeps replace the coarse flux on a coarse-fine
 * face, so mass, momentum and energy are conserved to round-off.  With one
 * level this is rg_step, bit for bit.
 *
 * d_u (device, 8 n_oct x 5 doubles, key order) is advanced in place;
 * d_scratch is a second buffer of the same size whose contents are
 * overwritten (levels alternate between the two buffers, so no level is
 * copied between substeps; the coarsest level is copied back at the end).
 * d_acc: rg_corr_workspace_bytes(n_oct - level_begin[lmin + 1]) bytes (the
 * per-oct kernel sums each level's coarse-side fluxes over the two substeps
 * into it; t->d_corr is not used); NULL only when lmin == lmax.  form is RG_FP64 or
 * RG_MIXED; tune as for rg_step (the brick kernel serves the bricks of the
 * schedule, if t->sched is set).  Asynchronous on `stream`; the host walks
 * the level recursion, issuing 2^(l - lmin) updates of level l. */
rg_status rg_step_subcycled(const rg_tree *t, double *d_u, double *d_scratch, double *d_acc, double gamma, double cfl,
                            int form, unsigned flags, double *d_dt, const rg_tuning *tune, void *stream);

/* ---------------------------------------------------------------------- */
/* Refinement and de-refinement                                           */
/* ---------------------------------------------------------------------- */

/* Refinement criterion (the paper does not state one for its hydro tests):
 * a cell of level l < lmax is flagged when rho > rho_thresh (rho_thresh > 0)
 * or when, for one of its six face neighbours n, |rho_n - rho| / (rho_n +
 * rho) > grad_thresh (grad_thresh > 0); n is the same-level cell, else the
 * coarse cell under the missing oct, and on an outflow face the cell itself.
 * Split cells are tested with their restricted values. */
typedef struct rg_refine_params {
    double rho_thresh;
    double grad_thresh;
    int32_t lmax;        /* finest level allowed: cells of level >= lmax are never flagged */
    int32_t nsubgrid;    /* 2 (or 0): cell by cell; 4: every flag, of the criterion or the closure, is
                            widened to all 8 cells of its oct, so octs come in complete sibling groups
                            (4^3-cell blocks, the paper's nsubgrid = 4 grids, Sec. 2) */
} rg_refine_params;

/* Bytes of the workspace rg_refine needs for a tree of `capacity` octs. */
size_t rg_refine_workspace_bytes(int64_t capacity);

/* The flags rg_refine acts on, into d_flags[n_oct] (bit c of an oct's word
 * = its cell c): the criterion alone (closure 0) or closed for grading
 * (closure 1): a flagged cell of level l needs its 26 neighbours and itself
 * at level l, so the level-(l-1) cells under the octs holding them are
 * flagged, levels taken from the finest down.  Reads d_u (key order). */
rg_status rg_refine_flags(const rg_tree *t, const double *d_u, const rg_refine_params *p, int closure,
                          uint32_t *d_flags, void *stream);

/* One refinement / de-refinement of tree t (Sec. 2.2: refine, de-refine,
 * sort by level, Hilbert order inside a level), on the device:
 *   flags as rg_refine_flags(closure = 1);
 *   new tree: every oct of level lmin, every oct above whose father cell is
 *   flagged, and a new oct under every flagged cell that has none; octs under
 *   unflagged cells are dropped (their fathers hold the restricted values);
 *   new state in d_u_new (key order of the new tree): kept octs copy their
 *   cells, a new oct's 8 cells take its father cell's values (injection, so
 *   leaf sums of volume * U are unchanged);
 *   keys, one radix sort, level ranges, hash table and neighbour lists of the
 *   new tree, written into t's buffers; t->n_oct, t->lmax and
 *   t->level_begin are updated and t->sched is set to NULL (rebuild a
 *   schedule with rg_schedule_build if wanted).
 * Every per-oct buffer of t (keys, scratch keys, permutation, coordinates,
 * neighbour lists, father cells, son masks, correction buffer) and the hash
 * and sort workspaces must be sized for t->capacity octs (0: n_oct);
 * RG_EFULL, with t unchanged, if the new tree would not fit.  d_u and
 * d_u_new are 8 x capacity x 5 doubles and must not alias; d_ws is
 * rg_refine_workspace_bytes(capacity) bytes, 256-byte aligned.  Synchronises
 * `stream` twice (the new oct count and the level ranges are read back). */
rg_status rg_refine(rg_tree *t, const double *d_u, double *d_u_new, const rg_refine_params *p, void *d_ws,
                    size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------- */
/* Multigrid Poisson solver                                               */
/* ---------------------------------------------------------------------- */

/* V-cycles for Lap phi = f (Sec. 5), 7-point Laplacian with cell width
 * h_l = 2^-l, on a hierarchy held by tree t: levels lcoarse .. lfine all
 * complete (every cell below lfine split, 8^(l-1) octs on level l),
 * periodic.  d_phi, d_f, d_r are per-cell arrays over the whole tree (8
 * n_oct doubles, key order).  On entry d_phi and d_f hold the initial guess
 * and the right-hand side on level lfine (f must have zero mean); the other
 * levels' entries are overwritten.  A V-cycle on level l: nu1 red-black
 * Gauss-Seidel sweeps (a red pass over the cells whose coordinates sum to an
 * even number, then a black pass; phi = (sum of the six neighbours - h^2 f)
 * / 6), the residual r = f - Lap phi, restricted into level l-1's f as the
 * mean of a cell's 8 children, a correction on level l-1 from zero
 * (recursively; ncoarse sweeps on lcoarse), added to phi by trilinear
 * interpolation (weights 27, 9, 3, 1 over 64 from the 8 coarse cells around
 * the fine cell), then nu2 sweeps.  ncycles cycles are run. */
rg_status rg_mg_vcycles(const rg_tree *t, double *d_phi, double *d_f, double *d_r, int lfine, int lcoarse, int nu1,
                        int nu2, int ncoarse, int ncycles, void *stream);

/* r = f - Lap phi on one complete periodic level of t (as in a V-cycle). */
rg_status rg_mg_residual(const rg_tree *t, const double *d_phi, const double *d_f, double *d_r, int level,
                         void *stream);

/* The potential on one level of an AMR tree (Sec. 5: built level by level
 * with V-cycles; the Gauss-Seidel diagonal adjusted in cells the boundary
 * cuts, located with a signed-distance-like mask).  Tree t: periodic, with
 * keys and neighbour lists.  Level L's unknowns are the potentials of its
 * octs' cells; the equation is Lap phi = f with the 7-point Laplacian and
 * h = 2^-L.  A face neighbour outside the level lies in a level-(L-1) leaf
 * (the tree is graded); its value is the trilinear interpolation of level
 * L-1's potential at its centre (weights 27, 9, 3, 1 over 64 from the 8
 * nearest level-(L-1) cells), fixed during the solve.  Level L-1 is solved
 * before level L and is not changed by it.  On the coarsest level of a tree
 * (complete, periodic) no neighbour is outside and f must have zero mean.
 *
 * The V-cycle's coarse levels m = L-1 .. lcoarse hold the ancestors of level
 * L's octs.  mask = +1 on level L's cells; on a coarse cell the mean of its
 * 8 children's masks (-1 for a cell without children).  A coarse cell is
 * inside when its mask is positive.  The coarse correction e solves Lap e =
 * (restricted residual) with e = 0 on the boundary: for an inside cell i
 * with s the sum of its inside face neighbours and d the sum over outside
 * ones j (absent cells count m_j = -1) of (m_i - m_j) / m_i - 1, a
 * Gauss-Seidel update is e_i = (s - h^2 f_i) / (6 + d) and the residual
 * f_i - (s - (6 + d) e_i) / h^2; outside cells keep e = 0 and residual 0.
 * One V-cycle on level l: nu1 sweeps (a red pass over cells with even
 * coordinate sum, then black), the residual, restricted to level l-1 as the
 * mean of 8 children (summed pairwise in cell order), a correction on l-1
 * from zero (recursively; ncoarse sweeps on lcoarse, or on L itself when
 * lcoarse == L), added by trilinear interpolation to the inside cells (absent
 * coarse cells count 0), then nu2 sweeps.  Faces are summed in the order x-,
 * x+, y-, y+, z-, z+.  On a complete level the values are rg_mg_vcycles'.
 *
 * rg_mg_level_create builds the hierarchy of level `level` (coarse keys,
 * their hash table, same-level neighbour lists, father links and masks) in
 * one device allocation owned by the handle; synchronises `stream` once per
 * coarse level.  The handle is valid while t's octs are unchanged (checked:
 * RG_EINVAL otherwise).  Errors: RG_EINVAL for a tree that is not periodic, a
 * level outside the tree or without octs, lcoarse outside 1..level;
 * RG_EHIP on allocation failure (nothing is then allocated). */
typedef struct rg_mg_level rg_mg_level;
rg_status rg_mg_level_create(const rg_tree *t, int level, int lcoarse, rg_mg_level **out, void *stream);

/* h_octs[m] (m = 0 .. RG_MAX_LEVEL) = octs of level m in the hierarchy
 * (level L's own octs at m = L). */
rg_status rg_mg_level_counts(const rg_mg_level *h, int64_t *h_octs);

/* ncycles V-cycles on h's level.  d_phi, d_f: per-cell arrays over the whole
 * tree (8 n_oct doubles, key order).  On entry d_phi holds level L-1's
 * potential (read) and the initial guess on level L, which is updated in
 * place; d_f holds the right-hand side on level L.  No other entry of either
 * array is read or written.  Calls on one handle must not overlap (the
 * handle holds the coarse levels' work arrays). */
rg_status rg_mg_level_vcycles(rg_mg_level *h, const rg_tree *t, double *d_phi, const double *d_f, int nu1, int nu2,
                              int ncoarse, int ncycles, void *stream);

/* d_r (per-cell over the whole tree) = f - Lap phi on the cells of h's
 * level, with the same boundary values; other entries are not written. */
rg_status rg_mg_level_residual(const rg_mg_level *h, const rg_tree *t, const double *d_phi, const double *d_f,
                               double *d_r, void *stream);

/* Frees the handle and its device memory (NULL: nothing). */
rg_status rg_mg_level_destroy(rg_mg_level *h);

/* ---------------------------------------------------------------------- */
/* Many independent trees in one graph launch                             */
/* ---------------------------------------------------------------------- */

/* The per-step phases of Table 1 (compute dt, godunov, set unew, upload) for
 * many independent trees at once.  This batched form is an addition of this
 * library, not a scheme of the paper: it fills the GPU with many small
 * boxes, each keeping its own time step.  Each phase of a step is one
 * persistent kernel looping over a work list that spans every tree: hash
 * rebuild and neighbour lists (with RG_STEP_REBUILD), CFL dt per tree, the
 * hydro update of every level of every tree (bricks and per-oct groups as in
 * the tree's schedule), the coarse-fine corrections (six passes), and the
 * restriction (one pass per depth below each tree's finest level).  The
 * phases of all `nsteps` steps are captured into one HIP graph.
 *
 * Tree t alternates between its two state buffers: step s reads d_u0 when s
 * is even (d_u1 when odd) and writes the other one, so after an even number
 * of steps the result is in d_u0.  The time step of tree t at step s is
 * written to d_dt[s * ntree + t] (device, double[(nsteps + 1) * ntree]): the
 * first from a pass over the state, each later one folded into the previous
 * step's update (as rg_step's RG_STEP_CHAIN_DT), and row nsteps holds the
 * time step a following step would take.  A tree gives the same bits, state
 * and dt, as rg_step run on it alone with the same form and flags.
 *
 * Every tree needs a schedule (t->sched, rg_schedule_build) and a correction
 * buffer if it has more than one level; keys, level ranges, hash workspace
 * and neighbour lists must be current when the graph runs (flags may only be
 * 0 or RG_STEP_REBUILD).  The trees must not share any device buffer.  The
 * rg_tree and rg_batch_tree structs are read during this call only; the
 * device buffers they point to are used by every rg_batch_run.
 * tune: octs_per_group 2, 4 (default) or 8; no_bricks 1 runs every oct
 * through the per-oct body; no_groups 1 leaves complete sibling groups to
 * the per-oct body (the batched group kernel runs 256 threads); persistent
 * selects persistent grids.  Every choice gives the same bits.  Allocates one device table (work lists and
 * tree descriptors) and the graph; synchronises `stream` once. */
typedef struct rg_batch_tree {
    const rg_tree *tree;
    double *d_u0, *d_u1;       /* state buffers, 8 n_oct x 5 doubles each */
    double gamma, cfl;
} rg_batch_tree;

typedef struct rg_batch rg_batch;

rg_status rg_batch_create(const rg_batch_tree *trees, int ntree, int form, int nsteps, unsigned flags,
                          const rg_tuning *tune, double *d_dt, void *stream, rg_batch **out);

/* Launches the captured graph (all steps) on `stream`; asynchronous. */
rg_status rg_batch_run(rg_batch *b, void *stream);

/* Frees the graph and the device table; NULL is allowed.  The caller makes
 * sure no launch of the graph is still running. */
rg_status rg_batch_destroy(rg_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* RG_H */
