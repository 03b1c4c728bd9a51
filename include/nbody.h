/*
 * nbody.h -- C ABI of libnbody_hip.so, a GPU-resident (MI355X, gfx950)
 * Barnes-Hut gravity step after "Accelerated FDPS" (Iwasawa et al. 2019):
 * Morton keys, radix sort, octree, group-wise walk emitting 32-bit index
 * interaction lists (section 4.1), one multiwalk force launch over all
 * groups (section 3), and reuse of the lists over several steps (section
 * 4.2), with a kick-drift leapfrog in FP64.
 *
 * Conventions shared by every entry point
 *   - Every call returns an int status: NB_OK (0) or a negative nb_status.
 *     On error nothing of the caller's memory has been written beyond what
 *     the call documents, and nb_last_error() describes the failure.
 *   - The library owns all device memory it allocates; the caller owns every
 *     buffer it passes and keeps ownership (inputs are copied in, outputs are
 *     copied out).  Host pointers are plain CPU memory; where a call takes
 *     `on_device`, a non-zero value means the pointers are device pointers
 *     on the context's GPU (for example torch.Tensor.data_ptr()).
 *   - Particle arrays use the caller's ORIGINAL order unless a call says
 *     INTERNAL order.  Internally the particles are kept in the Morton order
 *     of the last tree build; list ids refer to that internal order.
 *   - Work is enqueued on the context's HIP stream (the one given in
 *     nb_config.stream, or a stream the library creates).  Calls that return
 *     data to host memory synchronise that stream.  The moment pass of a
 *     construction step runs on a second stream the library owns, forked
 *     from and joined back into the context's stream by events before any
 *     work that reads the moments, so everything enqueued on the context's
 *     stream afterwards is ordered after it.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nb_ctx nb_ctx;

typedef enum nb_status {
  NB_OK = 0,
  NB_ERR_INPUT = -1, /* bad argument: NULL, size, NaN/inf position, range */
  NB_ERR_OOM = -2,   /* device or host allocation failed */
  NB_ERR_LIST = -3,  /* a list id out of range or a list pool overflow */
  NB_ERR_STATE = -4, /* call order violated (e.g. REUSE_LIST before any
                        MAKE_LIST_FOR_REUSE, or no particles) */
  NB_ERR_HIP = -5    /* a HIP runtime call failed */
} nb_status;

/* Reuse modes of the paper's top-level force call (section 5): make lists
 * and discard them, make lists and keep them, or reuse the kept lists.
 * NB_REUSE_REFRESH and NB_REUSE_CHECK (extensions, need NB_FLAG_REFRESH)
 * reuse the kept lists but first walk again the lists of the groups that
 * the predictor flags, or that the exact staleness check flags (see
 * nb_compute_forces). */
typedef enum nb_mode {
  NB_MAKE_LIST = 0,
  NB_MAKE_LIST_FOR_REUSE = 1,
  NB_REUSE_LIST = 2,
  NB_REUSE_REFRESH = 3,
  NB_REUSE_CHECK = 4
} nb_mode;

typedef struct nb_config {
  double theta;    /* opening angle of the Barnes-Hut test (section 2); 0
                      opens every cell.  Must be >= 0. */
  double eps;      /* Plummer softening length, > 0 */
  double G;        /* gravitational constant */
  double ext_mass; /* fixed point mass at the origin added in kick-drift
                      (0 = none); unsoftened */
  int32_t n_leaf;  /* a cell holding more than n_leaf particles is split
                      (section 6.1 uses 16); 1..64 */
  int32_t n_grp;   /* largest particle group sharing one list (section 3,
                      Barnes' vectorisation); 1..65536 */
  int32_t order;   /* superparticle expansion: 1 monopole, 2 quadrupole */
  int32_t flags;   /* bit 0: record per-phase GPU timers (HIP events);
                      bit 1: run the reuse steps of nb_step from a captured
                      HIP graph; bit 2: per-group list refresh (below);
                      bit 3: persistent force launch (resident workgroups
                      pull work items from per-XCD counters) */
  int32_t k_max;   /* refresh mode: a list this many reuse steps old is
                      walked again; 1..65535 */
  double p_star;   /* refresh mode: a list whose predicted staleness
                      exceeds p_star is walked again; [0, 1] */
  double tau;      /* refresh mode: staleness tolerance of NB_REUSE_CHECK
                      (see nb_group_stale); >= 0 */
  int32_t tile_j;  /* force kernel tile: list entries staged in LDS per
                      round, 64, 128, 192 or 256 (a group chunk of n_i <= 32
                      particles sums it on 64 / n_i lane slices); 0 = the
                      default (192 monopole, 128 quadrupole).  Section 3's
                      multiwalk kernel, tile shape of this GPU's instance */
  int32_t waves_per_simd; /* force kernel occupancy the register allocation
                      aims at: 4, 6 or 8 waves per SIMD; 0 = 6.  Neither
                      changes which interactions are summed; the persistent
                      launch (bit 3) keeps its own shape */
  void* stream;    /* hipStream_t to launch on; NULL = the library's own */
} nb_config;

/* Phase ids of the per-phase timers (nb_get_timing). */
enum {
  NB_PH_ROOT = 0,  /* root cell: bounding cube                 */
  NB_PH_KEYS,      /* Morton keys                               */
  NB_PH_SORT,      /* radix sort of key-index pairs             */
  NB_PH_REORDER,   /* reorder particles into Morton order       */
  NB_PH_LINK,      /* octree cells, DFS order                   */
  NB_PH_MOMENTS,   /* multipole moments                         */
  NB_PH_GROUPS,    /* particle groups and their boxes           */
  NB_PH_WALK,      /* tree walk -> index interaction lists      */
  NB_PH_FORCE,     /* multiwalk force kernel                    */
  NB_PH_KICK,      /* kick-drift                                */
  NB_PH_GRAPH,     /* a reuse step replayed from a HIP graph     */
  NB_PH_REFRESH,   /* predictor inputs, perceptron, list refresh */
  NB_PH_COUNT
};

enum {
  NB_FLAG_TIMING = 1,
  NB_FLAG_GRAPH = 2,
  NB_FLAG_REFRESH = 4,
  NB_FLAG_PERSISTENT = 8,
  /* Lists that hold copies of the j-data instead of indices (the paper's
   * method G1, section 4.1 and its table of methods; kept for comparison
   * with the index lists, G2): every force evaluation first copies each list
   * entry, as an FP32 offset from its group's centre and its mass, into a
   * per-group contiguous array (16 bytes per entry), and the force kernel
   * reads that.  Same forces bit for bit.  Order 1 only, not with
   * NB_FLAG_REFRESH or NB_FLAG_PERSISTENT (NB_ERR_INPUT). */
  NB_FLAG_COPIED_LISTS = 16,
  /* Multipole moments (section 4.3, recomputed at every step) with one
   * launch per tree level, leaves first, as the level-by-level link order
   * suggests; without it they take two launches (subtrees of at most 512
   * cells per workgroup in LDS, then the cells above them by one workgroup
   * through a table of child ids).  Both form every sum in the same order
   * and precision: the moments, and so the forces, are the same bit for
   * bit.  Kept for that comparison. */
  NB_FLAG_LEVEL_MOMENTS = 32
};

/* Rebuild predictor: inputs per group and parameter count of the
 * 12-64-64-1 perceptron (tanh, tanh, logistic).  Parameter layout (floats):
 * W1[64][12] row-major, b1[64], W2[64][64] row-major, b2[64], w3[64], b3. */
enum { NB_MLP_NIN = 12, NB_MLP_NPARAM = 5057 };

/* ---- lifetime --------------------------------------------------------- */

/* Create a context on the current HIP device.  cfg is copied.  One context
 * is one particle system with its tree and lists, the state the paper's
 * top-level force call works on (section 5); the opening angle, softening,
 * leaf and group sizes are those of its measurements (section 6.1).
 * Errors: NB_ERR_INPUT (cfg out of range), NB_ERR_HIP, NB_ERR_OOM. */
int nb_create(const nb_config* cfg, nb_ctx** out);

/* Destroy a context and free its device memory (NULL is a no-op).  Section
 * 5: the library owns the tree and the saved lists; they die with it. */
void nb_destroy(nb_ctx* ctx);

/* Replace the configuration (theta, eps, n_leaf, n_grp, order, ...).
 * Invalidates the tree and the lists; particles are kept (a new opening
 * angle or group size needs a construction step, section 4.2).
 * Errors: NB_ERR_INPUT (cfg out of range). */
int nb_set_config(nb_ctx* ctx, const nb_config* cfg);

/* Copy in n particles: positions, velocities and masses (FP64, original
 * order, 7 arrays of n doubles).  1 <= n < 2^31.  These are the full
 * particle records of section 4.3 (FP), from which the interaction records
 * (EPI, EPJ) are derived on the device; the caller keeps ownership of the
 * arrays.  Invalidates the tree and the lists (section 5: particles may not
 * change while a list is reused).
 * Errors: NB_ERR_INPUT (NULL, n out of range), NB_ERR_OOM. */
int nb_set_particles(nb_ctx* ctx, int64_t n, const double* x,
                     const double* y, const double* z, const double* vx,
                     const double* vy, const double* vz, const double* m,
                     int on_device);

/* Not in the paper (batching of independent systems, an extension; each
 * system is the paper's single system of section 4.3).
 * Split the particles into independent systems: system s is particles
 * [off[s], off[s + 1]) of the original order (off holds n_sys + 1 values,
 * off[0] = 0, off[n_sys] = n, every system non-empty).  Each system gets its
 * own root cell, tree, groups and lists and feels only its own particles;
 * all systems share every kernel launch.  nb_set_particles resets to one
 * system.  Invalidates the tree and the lists.
 * Errors: NB_ERR_STATE (no particles), NB_ERR_INPUT (bad offsets). */
int nb_set_systems(nb_ctx* ctx, int64_t n_sys, const int64_t* off);

/* ---- the step ----------------------------------------------------------
 * Construction step (section 4.3): root cell, Morton keys, radix sort,
 * reorder, link, moments, groups.  Particles move into Morton order.
 * Errors: NB_ERR_STATE (no particles), NB_ERR_INPUT (a non-finite position),
 * NB_ERR_OOM, NB_ERR_HIP. */
int nb_build_tree(nb_ctx* ctx);

/* Group-wise tree walk emitting index interaction lists (sections 4.1 and
 * 4.3).  NB_MAKE_LIST keeps them for the current positions only,
 * NB_MAKE_LIST_FOR_REUSE also keeps them for later NB_REUSE_LIST steps;
 * NB_REUSE_LIST is accepted when reusable lists exist and does nothing.
 * Requires a tree built on the current positions (NB_ERR_STATE). */
int nb_make_lists(nb_ctx* ctx, nb_mode mode);

/* The paper's top-level force call (section 5).  NB_MAKE_LIST and
 * NB_MAKE_LIST_FOR_REUSE run nb_build_tree, nb_make_lists(mode) and the
 * force kernel.  NB_REUSE_LIST (section 4.2) recomputes the moments of the
 * frozen tree from the current positions and runs the force kernel on the
 * kept lists; particles are not re-sorted.  Forces (acceleration including
 * G, and potential excluding the self term) stay on the device until read.
 * NB_REUSE_REFRESH does the same, and between moments and force kernel
 * computes the predictor inputs of every group (nb_group_features), runs
 * the perceptron and walks again every group with p > cfg.p_star or
 * age >= cfg.k_max, without synchronising with the host.  In refresh mode
 * each group's lists sit in a slot with room for three times the
 * constructed length plus the mean list length, and each of the 4 lanes of
 * its walk has room for twice its tokens at construction plus 32; a
 * walked-again list replaces the kept one in place when it fits both,
 * otherwise the group keeps its list and age, and is counted in info[15]
 * (nb_get_info).
 * NB_REUSE_CHECK does the same with the exact staleness check at tolerance
 * cfg.tau (nb_group_stale) in place of the predictor.
 * Errors: NB_ERR_STATE (REUSE_LIST without reusable lists or after
 * nb_set_particles; REUSE_REFRESH or REUSE_CHECK without NB_FLAG_REFRESH),
 * plus those of the stages. */
int nb_compute_forces(nb_ctx* ctx, nb_mode mode);

/* Kick-drift of the KDK leapfrog in FP64: v += (a + a_ext) * dt_kick, then
 * x += v * dt_drift, with a the last computed forces and a_ext the pull of
 * cfg.ext_mass at the origin.  Section 4.3: after the forces are written
 * back, the orbits of the particles are integrated (the paper does not name
 * the integrator; leapfrog is the reading used).  Requires computed forces
 * (NB_ERR_STATE).  Invalidates the tree for new lists; kept lists stay
 * reusable (section 4.2).  Errors: NB_ERR_INPUT (non-finite step). */
int nb_kick_drift(nb_ctx* ctx, double dt_kick, double dt_drift);

/* One leapfrog step (section 4.3: integrate, then the next force call with
 * its reuse mode, section 5): nb_kick_drift(dt_kick, dt_drift) then
 * nb_compute_forces(mode).  With NB_FLAG_GRAPH, the first NB_REUSE_LIST step
 * after a construction step captures kick-drift, moments and force kernel
 * into a HIP graph on the context's stream, and later reuse steps with the
 * same time steps replay it (one launch per step); a construction step, a
 * new configuration, another reuse mode or other time steps drop the graph.
 * In refresh mode (NB_FLAG_REFRESH) NB_REUSE_REFRESH and NB_REUSE_CHECK
 * steps are captured and replayed the same way (predictor or check,
 * selection, walk and list refresh all run on the device).  Results are the
 * same as without the flag.  Errors: those of the two calls. */
int nb_step(nb_ctx* ctx, nb_mode mode, double dt_kick, double dt_drift);

/* ---- readback (synchronises the stream) --------------------------------
 * Section 5: the retrieve step copies the results back to the caller's
 * particles.  internal = 0: original order; 1: internal (Morton) order.
 * Errors: NB_ERR_STATE (nothing computed), NB_ERR_INPUT (NULL). */
int nb_get_forces(nb_ctx* ctx, double* ax, double* ay, double* az,
                  double* pot, int internal);
int nb_get_state(nb_ctx* ctx, double* x, double* y, double* z, double* vx,
                 double* vy, double* vz, int internal);

/* Sizes and counters of the tree and lists (the quantities of section 6.1:
 * <n_i> = n / groups, <n_list> = (EPJ + SPJ entries) / groups).
 * info[0] n, [1] cells, [2] groups, [3] EPJ entries, [4] SPJ entries,
 * [5] interactions of the current lists (sum over groups of
 * n_i * (n_epj + n_spj)), [6] force evaluations so far, [7] total
 * interactions evaluated so far, [8] root exponent k of system 0, [9] force
 * work items, [10] systems, [11] groups whose lists the last force call
 * refreshed, [12] refreshed groups so far, [13] superparticle interactions
 * of the current lists (sum over groups of n_i * n_spj), [14] superparticle
 * interactions evaluated so far, [15] groups whose walked-again list did not
 * fit its slot in the last force call (they kept their lists), [16] the same
 * summed over force calls.  info must hold 17 values.  In refresh mode the
 * list sizes and these counts are kept on the device (a refresh changes the
 * lists without the host) and this call synchronises the stream to read
 * them. */
int nb_get_info(nb_ctx* ctx, int64_t* info);

/* Root corner lo[3] and exponent k of the last tree (side 2^k); with
 * several systems, those of system 0.  Section 4.3: the root cell is set
 * from the particle positions. */
int nb_get_root(nb_ctx* ctx, double* lo, int32_t* k);

/* Root corners (3 per system) and exponents (1 per system); section 4.3
 * root cell, one per independent system. */
int nb_get_roots(nb_ctx* ctx, double* lo3, int32_t* k);

/* Sorted keys (n) and, for each sorted position, the ORIGINAL index of the
 * particle there (n).  Section 4.3 steps 1-3: Morton keys, their sort and
 * the reorder of the particles. */
int nb_get_keys(nb_ctx* ctx, uint64_t* key, uint32_t* orig);

/* Section 4.3 step 4 (link): the tree cells.
 * Cell arrays in DFS pre-order (system after system), each of length
 * info[1]; any may be NULL.  The parent of a root is 0xFFFFFFFF; skip = id
 * after the subtree; ctr3 = geometric centres (3 per cell). */
int nb_get_cells(nb_ctx* ctx, uint8_t* level, uint32_t* begin,
                 uint32_t* count, uint32_t* parent, uint32_t* skip,
                 uint8_t* leaf, double* ctr3);

/* Moments per cell (section 4.3: multipole moments, recomputed every step):
 * mass, centre of mass (3), second moments about the centre of mass (6: xx
 * yy zz xy xz yz).  Any may be NULL. */
int nb_get_moments(nb_ctx* ctx, double* mass, double* com3, double* quad6);

/* Groups (length info[2]; section 2, Barnes' grouping of particles that
 * share one list): cell id, first particle, count, tight box lo3/hi3 and
 * centre ctr3 (3 per group).  Any may be NULL. */
int nb_get_groups(nb_ctx* ctx, uint32_t* cell, uint32_t* begin,
                  uint32_t* count, double* lo3, double* hi3, double* ctr3);

/* Lists in CSR form (section 4.1: indices of EPJ and SPJ instead of their
 * copies): epj_off/spj_off hold info[2]+1 offsets, epj/spj hold
 * info[3]/info[4] ids (EPJ = internal particle positions, SPJ = cell ids),
 * ascending within each group.  Any may be NULL.  (In refresh mode the
 * lists sit in per-group slots on the device and are packed here.) */
int nb_get_lists(nb_ctx* ctx, int64_t* epj_off, uint32_t* epj,
                 int64_t* spj_off, uint32_t* spj);

/* Install caller-made index lists for the current tree: the dispatch step
 * with indirect addressing of section 5 (at a construction step the index
 * lists are sent to the accelerator and saved there; reuse steps use the
 * saved lists) and the index lists of section 4.1.  Same CSR layout as
 * nb_get_lists: epj_off and spj_off hold n_groups + 1 offsets (from 0,
 * non-decreasing, ending at n_epj and n_spj), epj holds n_epj internal
 * particle slots, spj holds n_spj cell ids; any order within a group.
 * Host arrays, or device arrays on the context's GPU when on_device != 0;
 * the caller keeps ownership (they are copied).  Before any kernel indexes
 * with them, one device pass reads the offsets and one the ids and checks
 * them against n and the cell count; a failure returns NB_ERR_LIST and
 * leaves no lists installed.  On success the lists are reusable: the next
 * nb_compute_forces(NB_REUSE_LIST) evaluates them (moments refreshed, as at
 * any reuse step).  They stay until the next tree build or list walk.
 * Synchronises the stream twice.
 * Errors: NB_ERR_STATE (no tree, or refresh mode, whose per-list walk state
 * uploaded lists do not carry), NB_ERR_INPUT (n_groups differs from the
 * tree's, NULL arrays, negative totals), NB_ERR_LIST, NB_ERR_OOM,
 * NB_ERR_HIP. */
int nb_upload_lists(nb_ctx* ctx, int64_t n_groups, const int64_t* epj_off,
                    int64_t n_epj, const uint32_t* epj,
                    const int64_t* spj_off, int64_t n_spj,
                    const uint32_t* spj, int on_device);

/* Per-phase time, in the phases of the paper's breakdown of a step (table
 * of section 6.1).
 * Accumulated GPU milliseconds per phase (NB_PH_COUNT values) and the
 * number of timed intervals per phase (may be NULL), since the last reset;
 * needs cfg.flags bit 0.  reset != 0 clears the counters after reading. */
int nb_get_timing(nb_ctx* ctx, double* ms, int64_t* calls, int reset);

/* ---- short-range interactions ----------------------------------------
 * Section 2: short-range interactions (SPH) use the same group-wise tree
 * walk with a cell-opening criterion other than the opening angle;
 * section 4.2: their lists are kept over several steps.
 *
 * Neighbour lists for the search radius h_list over every group of the
 * current tree: a cell that holds the group is opened; any other cell when
 * its cube overlaps the group's tight box grown by h_list on every side
 * (on each axis the gap from the box to the cell's centre is at most half
 * the side plus h_list, FP64), and is skipped with its subtree otherwise;
 * an opened leaf adds its particles (internal slots, DFS order).  Every
 * particle within h_list of a member is on the member's group list, the
 * member included.  The lists stay valid through kick-drift steps (the
 * particle order is kept) until the next tree build: built with
 * h_list = h (1 + s), they hold every pair within h while no particle has
 * moved more than s h / 2 since.  Timed as the walk phase.
 * Errors: NB_ERR_INPUT (h_list negative or not finite), NB_ERR_STATE (no
 * tree of the current positions), NB_ERR_OOM, NB_ERR_HIP. */
int nb_neighbour_lists(nb_ctx* ctx, double h_list);

/* SPH density on the neighbour lists at the current positions:
 * rho_i = sum over the list of i's group of m_j W(|x_i - x_j|, h), W the
 * cubic spline of compact support h, W(r, h) = 8 / (pi h^3) w(r / h),
 * w(q) = 1 - 6 q^2 + 6 q^3 (q <= 1/2), 2 (1 - q)^3 (1/2 < q <= 1), 0
 * beyond; FP32 offsets from the group centre and FP32 sums, as in the force
 * kernel.  Timed as the force phase.
 * Errors: NB_ERR_STATE (no neighbour lists), NB_ERR_INPUT (h <= 0 or
 * h > h_list of the lists). */
int nb_sph_density(nb_ctx* ctx, double h);

/* The densities (n values; internal as for nb_get_forces); synchronises.
 * Errors: NB_ERR_STATE (no density computed), NB_ERR_INPUT (NULL). */
int nb_get_density(nb_ctx* ctx, double* rho, int internal);

/* The neighbour lists: n_entries (may be NULL) gets the total entry
 * count; off (n_groups + 1 values) and ids (n_entries values, internal
 * slots) may be NULL.  Synchronises.  Errors: NB_ERR_STATE (no lists). */
int nb_get_neighbour_lists(nb_ctx* ctx, int64_t* n_entries, int64_t* off,
                           uint32_t* ids);

/* ---- per-group list refresh (NB_FLAG_REFRESH) --------------------------
 * An extension of the list reuse of section 4.2, which keeps every list for
 * a fixed number of steps.  Cells keep their particle ranges between
 * construction steps; in every opening test of a refresh mode walk, the
 * geometric centre of a cell is moved by the displacement of its FP64
 * centre of mass since the construction step, so that a rigid motion stales
 * no list, and the cell's side becomes twice the largest per-axis distance
 * from that centre to the box of its current particles when that is larger
 * (a cell whose particles spread is opened sooner).  At construction the
 * shift is zero and the side the geometric one, so construction lists are
 * unchanged.
 * A group's list is stale (at tolerance tau >= 0) when one of its
 * superparticles fails the opening test at the relaxed angle theta (1 + tau)
 * from the group's current tight box; particles are exact and cells that a
 * fresh walk would accept higher up only cost work, so neither makes a list
 * stale.  Per group the library keeps the box, the cell shift
 * and the opening-test slacks of the walk that made its list, and the
 * list's age (reuse steps since that walk).  The calls below describe the
 * state of the last force computation (NB_ERR_STATE after a drift, without
 * the flag, or without reusable lists). */

/* The 12 predictor inputs per group, row-major [groups][12] FP32.  With s
 * the side of the group's cell, (lo, hi) its current box, (lo0, hi0), tau0,
 * sa, so the box, cell shift and slacks of the walk that made its list,
 * dtau = (current shift of the group's cell) - tau0:
 *   e_a = max(|lo_a - lo0_a - dtau_a|, |hi_a - hi0_a - dtau_a|), E = |e|,
 *   B = |dtau|, grow = max_a max(0, (hi - lo)_a - (hi0 - lo0)_a),
 *   f0 = min(age, k_max) / k_max, f1..f4 = log1p of E/sa, E/so, B/sa, B/so,
 *   f5 = log1p(E/s), f6 = log1p(B/s), f7 = log1p(sa/s), f8 = log1p(so/s),
 *   f9 = log1p(grow/s), f10 = log2(n_i)/6, f11 = log2(1 + list length)/16,
 * ratios capped at 1e6 (x/0 = cap, 0/0 = 0); computed in FP64, stored
 * FP32.  feat may be NULL (kept on the device for the predictor). */
int nb_group_features(nb_ctx* ctx, float* feat, int on_device);

/* Staleness labels at tolerance tau: stale[g] = 1 when a superparticle of
 * the kept list fails the opening test at angle theta (1 + tau) from the
 * group's current box and the cell's current centre (a check that changes
 * nothing); label[g] the same as 0.0 / 1.0.  Either may be NULL.
 * Errors: NB_ERR_INPUT (tau < 0 or not finite, theta = 0). */
int nb_group_stale(nb_ctx* ctx, double tau, uint8_t* stale, float* label,
                   int on_device);

/* Walk again the lists of the n_sel groups listed in sel (host array of
 * ascending group ids) with their current boxes and centres; other lists
 * are kept.  Sets those groups' box, shift, slacks and age (0).  When a new
 * list does not fit its group's room (see nb_compute_forces), the rooms of
 * those groups grow to twice the new list (every list moves to its new
 * slot) and the selection is walked again; a list that still does not fit
 * is not installed: that group keeps its list and state, and the call
 * returns NB_ERR_LIST after installing the others.  Synchronises the
 * stream.
 * Errors: NB_ERR_INPUT (ids not ascending or out of range), NB_ERR_LIST. */
int nb_refresh_lists(nb_ctx* ctx, int64_t n_sel, const int64_t* sel);

/* Slacks sa, so (FP64, +inf when no such cell) and ages per group; any may
 * be NULL.  sa = smallest |box - centre| - rcrit over accepted cells,
 * so = smallest rcrit - |box - centre| over opened cells not holding the
 * group, of the walk that made the list. */
int nb_get_group_state(nb_ctx* ctx, double* sa, double* so, int32_t* age);

/* The side each cell has in the opening test now (info[1] values, FP64). */
int nb_get_cell_sides(nb_ctx* ctx, double* side);

/* Not in the paper (the learned predictor of list staleness, an extension
 * of the fixed reuse interval of section 4.2).
 * Perceptron weights (host, NB_MLP_NPARAM floats).  Setting them clears the
 * Adam state.  A context starts with zero weights (p = 1/2). */
int nb_mlp_set(nb_ctx* ctx, const float* w, int64_t nw);
int nb_mlp_get(nb_ctx* ctx, float* w, int64_t nw);

/* p[i] = predicted staleness of input row x[i] (n rows of 12). */
int nb_mlp_forward(nb_ctx* ctx, int64_t n, const float* x, float* p,
                   int on_device);

/* Mean weighted cross-entropy over n rows, -(1/n) sum [w y log p +
 * (1 - y) log(1 - p)] with w = pos_weight > 0, and its gradient
 * (NB_MLP_NPARAM floats); loss is a host float; either may be NULL. */
int nb_mlp_grad(nb_ctx* ctx, int64_t n, const float* x, const float* y,
                float pos_weight, float* loss, float* grad, int on_device);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid
 * hipMalloc.  The same gradient and loss as nb_mlp_grad, from the same
 * kernels, with no allocation and no host synchronisation: x (n rows of 12),
 * y (n), grad (NB_MLP_NPARAM floats) and loss (1 float, may be NULL) are
 * device arrays on the context's GPU, and the work is only enqueued on the
 * context's stream (results are there once the stream reaches it).  The
 * per-sample activations and partial sums live in one static array per GPU
 * of about 8.2 MiB (1 <= n <= NB_MLP_STATIC_MAX_ROWS), held until the
 * process ends and shared by every context on that GPU: calls whose work
 * overlaps on one GPU (other streams, other contexts, other host threads)
 * race on it; calls on one stream are ordered and do not.  Nothing in the
 * array has to start at zero (each call writes what it reads).
 * Errors: NB_ERR_INPUT (n out of range, NULL x, y or grad, pos_weight <= 0),
 * NB_ERR_STATE (no weights: set them first with nb_mlp_set, which
 * allocates), NB_ERR_HIP. */
enum { NB_MLP_STATIC_MAX_ROWS = 8192 };
int nb_mlp_grad_static(nb_ctx* ctx, int64_t n, const float* x, const float* y,
                       float pos_weight, float* loss, float* grad);

/* One Adam step (Kingma and Ba) on the weights with gradient grad (NULL =
 * the last nb_mlp_grad gradient); the step counter starts at 1 after
 * nb_mlp_set. */
int nb_mlp_adam(nb_ctx* ctx, const float* grad, float lr, float beta1,
                float beta2, float eps, int on_device);

/* epochs passes over the n rows in order, in batches of `batch` rows, one
 * Adam step (beta 0.9, 0.999, eps 1e-8) per batch, all on the GPU; loss
 * (host, may be NULL) = the loss over all rows after training. */
int nb_mlp_train(nb_ctx* ctx, int64_t n, const float* x, const float* y,
                 int on_device, int epochs, int64_t batch, float lr,
                 float pos_weight, float* loss);

/* Description of the last error on this context ("" if none).  The paper
 * specifies no error handling (its library is C++ templates); every entry
 * point here returns a status instead. */
const char* nb_last_error(const nb_ctx* ctx);

/* Library version string (no paper counterpart). */
const char* nb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NBODY_H */
