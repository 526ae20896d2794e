/*
 * hines.h -- C-ABI of the MI355X batched Hines solver (libhines.so).
 *
 * The library solves, for every cell (neuron) of a forest, the linear system
 * A x = b of one implicit-Euler step of the discretised cable equation
 * (F. Huber, "Efficient Tree Solver for Hines Matrices on the GPU", §1, the
 * discrete system following the cable equation).  A is symmetric and strictly
 * diagonally dominant, so elimination needs no pivoting.  The solve is the
 * Hines algorithm (§2, Listing 2): backward elimination from the leaves to the
 * root through the parent array, a root solve, forward substitution from the
 * root to the leaves, carried out level-synchronously with one lane per branch
 * (§3) on a branch-to-lane assignment computed once at setup (§4-§6).
 *
 * Numbering (the "user numbering"), matching §2:
 *   - cell c owns compartments [cell_offsets[c], cell_offsets[c+1]);
 *   - the first compartment of a cell is its root and has parent -1;
 *   - every other compartment i has cell_offsets[c] <= parent[i] < i.
 * Matrix values:
 *   - diag[i]  = A[i][i];
 *   - upper[i] = A[i][parent[i]] = A[parent[i]][i], the signed entry (the
 *     negative edge conductance for the cable matrix); upper[root] is ignored.
 *
 * Conventions of every call:
 *   - Errors are return codes; nothing is thrown across the ABI.  A message for
 *     the last error of the calling thread is available from hines_last_error.
 *   - Device pointers are owned by the caller and are never retained or freed.
 *   - Device work is asynchronous on the given stream (a hipStream_t; NULL is
 *     the default stream).  Launch failures are reported as HINES_ERR_HIP; a
 *     fault inside a kernel surfaces at the caller's next synchronisation.
 *   - A plan may be used by one stream at a time.
 */
#ifndef HINES_H
#define HINES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hines_plan hines_plan; /* opaque, owned by the library */

typedef enum hines_status {
  HINES_OK = 0,
  HINES_ERR_NULL = 1,          /* a required pointer is NULL */
  HINES_ERR_BAD_OFFSETS = 2,   /* cell_offsets not 0 < ... < n, or sizes out of range */
  HINES_ERR_BAD_PARENT = 3,    /* a root's parent is not -1, or parent[i] outside [cell start, i) */
  HINES_ERR_BAD_BRANCHES = 4,  /* branch layout invalid (see hines_setup) */
  /* 5 is not used: a level wider than a group is walked by lanes that take
     several branches each, so no width is ever refused */
  HINES_ERR_NCELLS = 6,        /* ncells differs from the plan's */
  HINES_ERR_OPTION = 7,        /* an option value is out of range */
  HINES_ERR_OOM = 8,           /* host or device allocation failed; the environment variable
                                  HINES_DEVICE_BYTE_CAP (bytes) caps the device memory the
                                  library holds, so that this path can be forced */
  HINES_ERR_HIP = 9,           /* a HIP runtime call or kernel launch failed */
  HINES_ERR_TOO_BIG = 10,      /* a group does not fit the device's LDS */
  HINES_ERR_NOT_SDD = 11,      /* hines_check_matrix: a row is not strictly diagonally dominant */
  HINES_ERR_STATE = 12         /* the plan was built host_only, or similar misuse */
} hines_status;

/* Setup options (paper §4-§6).  Obtain defaults from hines_default_options. */
typedef struct hines_options {
  int32_t rebalance_root;     /* §6: re-root each cell at its tree centre (0/1)            */
  int32_t split_branches;     /* §6: split branches longer than their level's average: 0 no,
                                 1 the average over all cells, 2 the average over the cells of
                                 one group of an intermediate packing (the per-block averages
                                 of the outlook, §8)                                         */
  int32_t group_width;        /* §3-§4: lanes per group; multiple of 64 in [64, 1024]      */
  int32_t cell_order;         /* §4 greedy packing order: 0 input order, 1 size descending  */
  int32_t max_group_unknowns; /* cap on compartments packed into one group; 0 = automatic   */
  int32_t host_only;          /* 1: build the tables only (no device upload, no solve)      */
  int32_t keep_tables;        /* 1: keep the exported tables for hines_get_table            */
  int32_t bitwise;            /* 1: IEEE divisions and unfused updates, so the solution equals
                                 the plain algorithm (§2 Listing 2) on the plan numbering bit
                                 for bit; 0 (default): reciprocal + fused multiply-add form   */
  int32_t level_sync;         /* 1: level-synchronous sweeps with a barrier per level (§3);
                                 0 (default): when every branch runs toward higher user indices
                                 and bitwise is 0, a static per-lane schedule computed at setup
                                 (each branch starts once its children are done; no barriers) */
  int32_t cell_lanes;         /* 1: hines_solve and hines_timestep run one lane per cell, the
                                 one-thread-per-matrix solver of §3 and §7 (§2's elimination in a
                                 depth-first order of each cell, 64 lanes of similar length per
                                 wave; a cell longer than 80% of the mean cell (cell_cut_percent)
                                 is cut into pieces on two to four lanes of one wave (at most
                                 cell_max_cuts + 1); elimination factors kept in a
                                 device scratch of 16 bytes per step owned by the plan).  Needs
                                 bitwise 0, cells of at most 65535 compartments and a stack need
                                 of at most 12 (HINES_ERR_TOO_BIG otherwise).  hines_solve_mixed
                                 keeps using the groups.
                                 2: hines_solve runs index-order cell lanes: the same solver,
                                 but each lane eliminates its piece of a cell in decreasing
                                 user index (children first by §2's numbering), so that a
                                 cell numbered level by level is read in long runs of whole
                                 memory lines; contributions to a parent that is not the next
                                 step wait in up to 26 LDS slots per lane (a lane that would
                                 need more walks depth-first); while a piece of a cell is
                                 longer than cell_cut_percent of the mean cell it is cut
                                 again, into at most cell_max_cuts + 1 pieces on adjacent
                                 lanes.  Runs start on 128-byte lines when the arrays do.
                                 Needs bitwise 0 and cells of at most 65535 compartments
                                 (HINES_ERR_TOO_BIG otherwise).  hines_timestep and the time
                                 loop (one solve per step) run on it too; the solver layout,
                                 hines_solve_stored32 and hines_timestep_assembled need
                                 cell_lanes 1 (HINES_ERR_STATE).
                                 0 (default): groups (§3-§4)                                 */
  int32_t resident;           /* 1: hines_solve runs the LDS-resident kernel: consecutive whole
                                 cells form a group of up to 1400 compartments (a larger cell is
                                 a group of its own; see res_pack); one wave stages the group's
                                 d, u, b into LDS once, eliminates every compartment after its
                                 children (§2) along root-ward paths that setup cuts into chunks
                                 of 8 steps and schedules on the wave's 64 lanes (§3-§4), and
                                 stores x.  With rebalance_root each cell is eliminated from
                                 its tree centre (§6), the couplings on the path from the old
                                 root moved at staging; x is still written in the user
                                 numbering.  Needs bitwise 0, cell_lanes 0 and every cell's
                                 image within LDS (up to about 6,100 compartments;
                                 HINES_ERR_TOO_BIG otherwise).  The other calls keep using the
                                 groups.                                                     */
  /* Tuning of the cell-lane and resident tables (0 selects the default): */
  int32_t cell_cut_percent;   /* cell lanes: cells longer than this percentage of the mean cell
                                 are cut into pieces on several lanes (default 80)           */
  int32_t cell_max_cuts;      /* cell lanes: at most this many cut-off subtrees per cell, 1..3
                                 (default 3)                                                 */
  int32_t res_pack;           /* resident: consecutive cells share a group while it holds at
                                 most this many compartments, 1..16000 (default 1400)       */
  int32_t level_balance;      /* 1: §8 outlook: a cell that overflows a level of the open group
                                 may move subtrees one level down (the smallest first) until
                                 every level fits; the level of a branch is then its step in the
                                 level-synchronous sweeps, deeper than its parent's            */
  int32_t reserved[1];        /* must be 0 */
} hines_options;

/* Plan summary. */
typedef struct hines_plan_info {
  int64_t n, ncells, nbranches, ngroups, nsegments;
  int32_t max_level;          /* deepest branch level (root branch = 0) */
  int32_t nclasses;           /* LDS size classes (kernel launches per solve) */
  int64_t device_table_bytes; /* device memory held by the plan */
  int64_t max_group_lds_bytes;
  int32_t kernel;             /* 0 level-synchronous, 1 flow (static step schedule), 2 bitwise,
                                 3 cell lanes, 4 LDS-resident, 5 index-order cell lanes       */
  int32_t max_makespan;       /* flow plans: longest schedule, in chunk steps; cell-lane plans:
                                 chunks per sweep of the longest wave; resident plans: steps
                                 per sweep of the longest group                              */
  int64_t workspace_groups;   /* groups too large for LDS, solved from a global workspace */
} hines_plan_info;

typedef struct hines_timeloop hines_timeloop; /* opaque: a captured multi-step graph */

/* Table ids for hines_get_table (all exported as int64). */
enum {
  HINES_TABLE_NODE_PLAN = 0,         /* [n]  plan index of each user compartment              */
  HINES_TABLE_BRANCHES = 1,          /* [nb*8] per plan branch: cell, level, first user index,
                                        direction (+1/-1), length, parent branch (-1), group,
                                        breadth-first rank in its cell                         */
  HINES_TABLE_U_SRC = 2,             /* [n] per plan index: the user index whose upper[] holds
                                        its coupling to the plan parent (-1 for roots)         */
  HINES_TABLE_GROUP_OFFSETS = 3,     /* [ngroups+1]                                            */
  HINES_TABLE_GROUP_CELLS = 4,       /* [ncells] cells of the groups, packing order            */
  HINES_TABLE_GROUP_SEG_OFFSETS = 5, /* [ngroups+1] first (group, level) segment of each group */
  HINES_TABLE_SEG_OFFSETS = 6,       /* [nseg+1] first lane of each segment                    */
  HINES_TABLE_LANES = 7,             /* [nb] plan branch ids in (group, level, lane) order     */
  /* Step schedule of the flow kernel (plans with flow, see hines_plan_info.kernel == 1): */
  HINES_TABLE_FLOW_GROUPS = 8,       /* [ngroups*6] step_off, pos_off, aux_off, nsteps, nelem,
                                        npush per group (nsteps 0: group solved elsewhere)  */
  HINES_TABLE_FLOW_MASKS = 9,        /* [2*steps] per step: active-lane and push-lane masks
                                        (64-bit patterns stored in int64)                    */
  HINES_TABLE_FLOW_POS = 10,         /* [elements] LDS position of each element of a group's
                                        staging order; 0x8000 marks a cell root              */
  HINES_TABLE_FLOW_AUX = 11,         /* [pushes] position receiving each push, step order     */
  /* Cell-lane plans (hines_plan_info.kernel == 3): 64 lanes per wave, chunks of K = 16
     steps (K * 64 entries per chunk).                                                       */
  HINES_TABLE_CELL_WAVES = 12,       /* [nwaves*3] first chunk, chunks per sweep, cells       */
  HINES_TABLE_CELL_LANES = 13,       /* [nwaves*64] cell of each lane, -1 if empty            */
  HINES_TABLE_CELL_POS = 14,         /* [chunks*K*64] per chunk, lane j, slot r: position of
                                        element (j % K) of lane ((64 / K) r + j / K)'s walk,
                                        relative to its cell's first compartment, in backward
                                        step order; 65535 for padding                         */
  HINES_TABLE_CELL_FLAGS = 15,       /* [chunks*K*64] per chunk, lane c, element e: flags
                                        1 tip, 2 pop, 4 push, 8 merge, 16 padding, 32 root,
                                        64 root of a cut-off subtree (its contribution leaves
                                        through mailbox c), 128 parent of such a root (takes
                                        the next mailbox of the lane's source list)           */
  HINES_TABLE_CELL_MBSRC = 16,       /* [nwaves*64] per lane: the mailbox (source lane) of each
                                        take, 6 bits each, in backward order in bits 0-31 and
                                        in forward order in bits 32-63; 0 without takes       */
  /* LDS-resident plans (hines_plan_info.kernel == 4).  Group image: slot s holds user index
     lo + s; slot nslot is a zero entry (d = 1, u = 0, b = 0).                                */
  HINES_TABLE_RES_GROUPS = 17,       /* [ngroups*16] lo, blob (16-byte units), nslot, staged
                                        slots, slot of the first compartment, compartments,
                                        chunks per sweep, blob units, cells, path records,
                                        slot-list entries, byte offsets of the records and of
                                        the slot lists in the blob, LDS class, steps per chunk,
                                        re-rooting pairs                                      */
  HINES_TABLE_CELL_RANGE = 18,      /* [nwaves*64] per lane: the steps q0 .. q1 - 1 of its walk
                                        (bits 0-31: q0, bits 32-63: q1); every other step of
                                        the lane is padding; 0 for empty lanes                */
  HINES_TABLE_RES_BLOB = 19,         /* [blob bytes / 2] the group blobs as 16-bit words: per lane
                                        its first record and its first slot-list entry (65 + 65
                                        words, 136 in all), the root slots padded to 8 words,
                                        the re-rooting pairs (slot, slot whose staged u becomes
                                        its coupling) padded to 8 words,
                                        the path records (first chunk, chunks, byte offset of
                                        the top's parent entry or 0xffff for a cell root, 0),
                                        each lane's records enclosed by idle records (65535, 0,
                                        0xffff, 0), then per lane one entry per active chunk:
                                        the byte offsets (slot * 8) of its steps, the path's
                                        bottom first (padding steps point at the zero entry) */
  /* Index-order cell-lane plans (hines_plan_info.kernel == 5), chunks of K = 8 steps.       */
  HINES_TABLE_SEQ_WAVES = 20,        /* [nwaves*3] first chunk, chunks, cells                  */
  HINES_TABLE_SEQ_LANES = 21,        /* [nwaves*64] cell of each lane (-1: empty); a cut cell
                                        holds lanes c (the rest) and c + 1 (the subtree)      */
  HINES_TABLE_SEQ_POS = 22,          /* [chunks*K*64] as HINES_TABLE_CELL_POS with K = 8       */
  HINES_TABLE_SEQ_CODE = 23,         /* [chunks*K*64] per chunk, lane c, element e: bits 0-4 the
                                        slot the step's contribution goes into (0: the next
                                        step takes it), bits 5-9 the slot the step reads (its
                                        other children's contributions; 0: none), 1024 no
                                        carry from the previous step, 2048 padding, 4096 root
                                        of the cut-off subtree (mailbox c), 8192 its parent
                                        (takes the mailbox of the source lane), 16384 first
                                        contribution into its slot, 32768 the cell root       */
  HINES_TABLE_SEQ_MBSRC = 24         /* [nwaves*64] as HINES_TABLE_CELL_MBSRC                  */
};

/* Fill *opt with the defaults: no re-rooting, no splitting, group_width 64,
 * input cell order, automatic cap, device upload, keep tables. */
void hines_default_options(hines_options* opt);

/* Build a plan (paper §4: "computed once during the setup phase"; §6: the
 * optional balancing and splitting passes run before the packing).
 *   parent[n], cell_offsets[ncells+1]: host arrays in the user numbering.
 *   branch_offsets[nbranches+1]: optional host array (NULL: branches are the
 *     maximal runs of consecutive compartments, §2).  If given it must run from
 *     0 to n, increase strictly, start a branch at every cell start, and have
 *     parent[i] == i-1 inside each branch.  Branches are further cut after any
 *     compartment that has a child outside its branch.  Ignored when
 *     rebalance_root is set.
 *   opt: NULL for defaults.
 * Host arrays are only read during the call.  The plan's device tables are
 * allocated on the current device.  On error *out is set to NULL.
 * The per-cell tables of cell-lane plans are built by host threads, as many
 * as the environment variable HINES_SETUP_THREADS says, else one per host
 * core (at most 16); the tables do not depend on the count. */
hines_status hines_setup(const int32_t* parent, int64_t n, const int64_t* branch_offsets,
                         int64_t nbranches, const int64_t* cell_offsets, int32_t ncells,
                         const hines_options* opt, hines_plan** out);

/* Solve A x = rhs for all cells in FP64 (paper §2 Listing 2, §3 level-
 * synchronous sweeps, §5 one read of each matrix entry per sweep).
 *   diag, upper, rhs, x: device arrays of n doubles in the user numbering.
 *   x may alias rhs; it must not alias diag or upper.
 *   ncells must equal the plan's cell count.
 * Inputs are not modified.  Asynchronous on stream. */
hines_status hines_solve(const hines_plan* plan, const double* diag, const double* upper,
                         const double* rhs, double* x, int32_t ncells, void* stream);

/* hines_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same cell-lane kernel (depth-first or index-order lanes) and results as
 * hines_solve, with its per-step factors (16 bytes per walk slot) kept in a
 * file-scope device array of 256 MiB (kStaticScratchBytes) instead of the
 * plan's own scratch.  The call launches one kernel and allocates or frees
 * nothing.  Each device holds one such array from the first hines_setup on it
 * until the process ends; every call on that device uses it, so calls that
 * overlap on one device (several streams, or host threads) race and must be
 * serialised by the caller.  The kernel writes every scratch slot it reads
 * within the same call, so nothing needs clearing.
 *   Cell-lane plans only, cell_lanes 1 or 2 (HINES_ERR_STATE otherwise).
 *   HINES_ERR_TOO_BIG if the plan's factors exceed the array (about 14 million
 *   compartments of C2-like cells).  Arguments as hines_solve; x may alias
 *   rhs.  Async on stream. */
hines_status hines_solve_noalloc(const hines_plan* plan, const double* diag, const double* upper,
                                 const double* rhs, double* x, int32_t ncells, void* stream);

/* FP32 storage, FP64 elimination (cell-lane plans only).  The matrix is the
 * FP32 one (diag32, upper32: device float arrays, user numbering); the kernel
 * widens each entry exactly on load and runs §2's elimination in FP64, so one
 * sweep solves A x = rhs to FP64 rounding and no refinement is needed: on this
 * hardware FP64 and FP32 vector arithmetic issue at the same rate, and the
 * FP32 storage only cuts the bytes of the matrix (24 instead of 32 bytes per
 * compartment, with rhs and x in FP64).  HINES_ERR_STATE on a plan without
 * cell lanes.  x may alias rhs.  Async on stream. */
hines_status hines_solve_stored32(const hines_plan* plan, const float* diag32, const float* upper32,
                                  const double* rhs, double* x, int32_t ncells, void* stream);

/* FP32 storage and elimination with FP64 refinement.  The matrix is the FP32
 * one (diag32, upper32: device float arrays, user numbering), widened exactly
 * where FP64 arithmetic is used; rhs and x are FP64.  Sweep 0 solves
 * A x = fl32(rhs) in FP32; each further sweep (up to `sweeps`, at most 8)
 * forms r = rhs - A x in FP64, solves A d = fl32(r) in FP32 and adds d to x
 * in FP64.  The group's matrix, rhs and solution stay in LDS across sweeps,
 * so HBM sees 24 bytes per compartment whatever the number of sweeps.
 * HINES_ERR_TOO_BIG if a group does not fit this kernel's LDS image (or, on a
 * cell-lane plan, the groups' 16-bit branch records: a cell-lane plan is
 * still built then, and only this call is refused).
 * x may alias rhs.  Async on stream. */
hines_status hines_solve_mixed(const hines_plan* plan, const float* diag32, const float* upper32,
                               const double* rhs, double* x, int32_t sweeps, int32_t ncells, void* stream);

/* One implicit-Euler step of the discrete cable system (paper §1: the
 * current is evaluated at the old step):
 *     A v_out = c * v_in + I,   A given by (diag, upper),
 * with I = i_inj (device array, per compartment, constant) when i_inj is
 * non-NULL, else I_i = noise_sigma * Z_i where Z_i is a standard normal drawn
 * from Philox4x32-10 (Salmon et al., SC'11) keyed by (noise_seed, 0) with
 * counter (i mod 2^32, i div 2^32, step, 0) for user index i, and turned into a
 * normal by Box-Muller on two 52-bit uniforms; noise_sigma == 0 and i_inj ==
 * NULL give I = 0.  The right-hand side is formed inside the solve kernels.
 * v_out may alias v_in (in-place update); no other aliasing.  Async on stream. */
hines_status hines_timestep(const hines_plan* plan, const double* diag, const double* upper, const double* c,
                            const double* v_in, double* v_out, const double* i_inj, double noise_sigma,
                            uint32_t noise_seed, uint32_t step, int32_t ncells, void* stream);

/* One implicit-Euler step whose matrix is assembled in the solve (paper §1:
 * the discrete cable equation, diagonal = capacitive term plus the
 * conductances meeting at the compartment), for models whose diagonal
 * changes every step through a linearised membrane current g (V - E):
 *     A v_out = c * v_in + ge,
 *     A_ii = c_i + g_i + a_i + sum_{k: parent[k] = i} a_k,   A_{i,parent(i)} = -a_i,
 * with the edge conductances given as upper = -a (upper[root] is ignored, as
 * in hines_solve), g and ge = g * E per compartment (device arrays, user
 * numbering).  The diagonal is formed while the cell-lane kernel eliminates,
 * so no diag array is written or read.  Cell-lane plans only
 * (HINES_ERR_STATE otherwise).  v_out may alias v_in.  Async on stream. */
hines_status hines_timestep_assembled(const hines_plan* plan, const double* g, const double* upper, const double* c,
                                      const double* ge, const double* v_in, double* v_out, int32_t ncells,
                                      void* stream);

/* Capture nsteps consecutive hines_timestep calls, updating v in place with
 * steps first_step .. first_step + nsteps - 1, into a HIP graph (captured on
 * a private stream; nothing runs during creation).  Each
 * hines_timeloop_launch replays the same steps on `stream`; the arrays are
 * bound at creation and must stay valid.  The plan must outlive the loop.
 * On a cell-lane plan (option cell_lanes) the loop allocates, at creation,
 * up to 40 bytes per walk slot (cell compartments plus padding) and each
 * launch factors A once (f = u / d' and 1 / d' per compartment), moves c, the
 * current and v into the lanes' walk order, runs the nsteps right-hand-side
 * sweeps there and writes v back in user order at the end: the result equals
 * nsteps hines_timestep calls bit for bit.  If that allocation fails, the
 * loop captures nsteps plain hines_timestep launches instead (same results);
 * hines_timeloop_destroy frees what was allocated.  On a plan with no compartments the
 * loop holds no graph and its launch does nothing (the arrays may be NULL). */
hines_status hines_timeloop_create(const hines_plan* plan, const double* diag, const double* upper,
                                   const double* c, double* v, const double* i_inj, double noise_sigma,
                                   uint32_t noise_seed, uint32_t first_step, int32_t nsteps, int32_t ncells,
                                   hines_timeloop** out);
hines_status hines_timeloop_launch(hines_timeloop* loop, void* stream);
hines_status hines_timeloop_destroy(hines_timeloop* loop);

/* Element-wise kernels of the adjoint of the time loop (paper §1: A is
 * symmetric, A = diag(c) + L(a) with L the weighted graph Laplacian of the
 * tree).  All arrays are device arrays in the user numbering; a[i] is the
 * conductance of the edge (i, parent[i]) (a[root] is ignored).  The first call
 * uploads the parent array and child lists of the plan.
 *   hines_assemble:   diag_i = c_i + a_i + sum_{k: parent[k]=i} a_k (children in
 *                     ascending order), upper_i = -a_i (0 at roots).
 *   hines_gather_roots: out[cell] = v[first compartment of cell].
 *   hines_adjoint_rhs:  mu = c * lam_next (lam_next may be NULL: 0), plus
 *                     g_roots[cell] at each cell's root.
 *   hines_adjoint_accumulate: grad_i += lam; grad_c += lam * (v_prev - v);
 *                     grad_a[i] += -(lam_i - lam_p)(v_i - v_p), p = parent[i]. */
hines_status hines_assemble(hines_plan* plan, const double* a, const double* c, double* diag, double* upper,
                            void* stream);
hines_status hines_gather_roots(hines_plan* plan, const double* v, double* out, void* stream);
hines_status hines_adjoint_rhs(hines_plan* plan, const double* c, const double* lam_next, const double* g_roots,
                               double* mu, void* stream);
hines_status hines_adjoint_accumulate(hines_plan* plan, const double* lam, const double* v, const double* v_prev,
                                      double* grad_a, double* grad_c, double* grad_i, void* stream);

/* The solver layout of a cell-lane plan (paper §7, Fig 7.1: the solver works
 * on a solver-specific data format; permutation kernels move data into it and
 * the solution out of it).  A compartment's slot is its step in the walk of
 * its lane: per (wave, chunk of 16 steps, pair of steps, lane) one 16-byte
 * unit of two doubles, so a wave instruction of the solve touches one
 * contiguous KiB.  Slots beyond a lane's walk (padding) hold a copy of the
 * cell's first compartment.
 *   hines_layout_size: *slots = doubles of one array in the layout (the
 *     padded step count of all waves times 64).
 *   hines_to_layout:   dst[slots] <- src[n] (user numbering), any array.
 *   hines_from_layout: dst[n] <- src[slots]; padding slots are not read.
 *   hines_solve_layout: A x = rhs with diag, upper, rhs and x all in the
 *     layout (device arrays of `slots` doubles); upper of a cell root and of
 *     padding is ignored.  x may alias rhs, not diag or upper.  Bytes moved:
 *     d, u, b read and x written once, plus a 16-byte round trip per slot
 *     through the plan's scratch (the factors between the two sweeps).
 * HINES_ERR_STATE on a plan without cell lanes.  src and dst must not alias.
 * Asynchronous on stream. */
hines_status hines_layout_size(const hines_plan* plan, int64_t* slots);
hines_status hines_to_layout(const hines_plan* plan, const double* src, double* dst, void* stream);
hines_status hines_from_layout(const hines_plan* plan, const double* src, double* dst, void* stream);
hines_status hines_solve_layout(const hines_plan* plan, const double* diag_l, const double* upper_l,
                                const double* rhs_l, double* x_l, int32_t ncells, void* stream);

/* Check that (diag, upper) is a matrix the solver is defined for (paper §1:
 * A is symmetric, which the storage of one coupling per edge guarantees, and
 * strictly diagonally dominant with a positive diagonal, so elimination
 * without pivoting keeps every pivot positive).  Row i passes when
 *     diag[i] > |upper[i]| (not for a root) + sum over children k of |upper[k]|,
 * the sum taken over the children in ascending index; a NaN entry fails.
 *   diag, upper: device arrays of n doubles in the user numbering.
 *   first_bad: NULL, or set to the smallest failing user index (-1 if none).
 * The first call uploads the plan's parent array and child lists.  The call
 * is synchronous: it returns after the check has run on `stream`.
 * HINES_ERR_NOT_SDD if some row fails, HINES_OK otherwise. */
hines_status hines_check_matrix(hines_plan* plan, const double* diag, const double* upper, int64_t* first_bad,
                                void* stream);

/* Summary counts of a plan. */
hines_status hines_plan_info_get(const hines_plan* plan, hines_plan_info* info);

/* Copy table `which` (HINES_TABLE_*) to host memory as int64.  With
 * host_out == NULL only *count is set.  capacity is in elements;
 * HINES_ERR_OPTION if too small, unknown id, or tables were not kept. */
hines_status hines_get_table(const hines_plan* plan, int32_t which, int64_t* host_out,
                             int64_t capacity, int64_t* count);

/* Free the plan and its device tables (synchronises the device first).
 * NULL is accepted. */
hines_status hines_destroy(hines_plan* plan);

/* Static description of a status code. */
const char* hines_status_str(hines_status s);

/* Message of the last failing call on this thread ("" if none). */
const char* hines_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HINES_H */
