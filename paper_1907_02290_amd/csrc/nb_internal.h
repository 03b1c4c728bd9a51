// nb_internal.h -- private declarations of libnbody_hip.so (gfx950).
// Shared by the library's own translation units only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/nbody.h"

namespace nb {

constexpr int kKeyBits = 21;   // bits per axis in a Morton key
constexpr int kMaxLevel = 21;  // deepest tree level
constexpr int kLevels = kMaxLevel + 1;
constexpr uint32_t kNone = 0xFFFFFFFFu;
// lanes per group of the gravity walk over many groups (2, 4 or 8)
constexpr int kSplitLanes = 4;
// Spare tokens of a refresh-walk lane beyond twice its construction count.
constexpr uint32_t kLaneSpare = 32;

// Root cell of the last construction step, resident on the device.
struct Root {
  double lo[3];
  double rcrit2[kLevels];  // (side_l / theta)^2 per level
  double rr;               // (1/theta)^2: rcrit2[l] = ldexp(rr, 2 (k - l))
  int32_t k;               // side of the root cube = 2^k
  int32_t bad;             // non-zero: a non-finite coordinate was seen
};

// One tree cell, 64-byte aligned so that a walk visit touches one line.
//   geo  = geometric centre (x, y, z) and (side / theta)^2 of its level
//   meta = first particle, one past the last, id after the subtree,
//          level | leaf << 8
//   aux  = parent id (kNone for the root), unused x3
struct __attribute__((aligned(64))) CellRec {
  double4 geo;
  uint4 meta;
  uint4 aux;
};

// The walk's view of a cell in 16 bytes (one load per visit):
//   x, y = integer coordinates of the cell at its level, packed as
//          qx | qy << 21 | qz << 42 over the 64 bits x | y << 32, and the
//          leaf flag in bit 31 of y
//   z    = id after the subtree
//   w    = level | particle count << 5 for leaves (saturated at
//          kWalkCountSat; the exact count is in CellRec), 0 otherwise
// The walk rebuilds the centre and (side / theta)^2 from these with the same
// FP64 operations as the tree build, so the opening test is unchanged.
constexpr uint32_t kWalkCountSat = (1u << 27) - 1u;

// Where a refresh-mode walk writes its per-slot counts and the state of the
// walk (opening-test slacks, cell shift): slot t is group t of a
// construction walk or group sel[t] of a refresh.  With n_dev the number
// of slots walked is read on the device (at most the launch's n_walk).
struct WalkOut {
  uint32_t* cnt_e;
  uint32_t* cnt_s;
  uint32_t* cnt_t;
  double* sa;
  double* so;
  double4* tau0;
  const uint32_t* n_dev;
};

// Device counters kept in nb_ctx::red (u64):
//   0 interactions of the current lists, 1 largest token count of one slab,
//   2 superparticle interactions of the current lists, 4 / 5 particle and
//   superparticle entries of the current lists, 6 / 7 groups refreshed and
//   groups whose refreshed list did not fit, in the last force call,
//   8 / 9 interactions and superparticle interactions evaluated, 10 / 11
//   groups refreshed and refreshes that did not fit, summed over force calls
//   (8-11: refresh mode, where every force call adds to them on the device).
enum {
  kRedInter = 0, kRedMaxTok = 1, kRedInterSpj = 2, kRedEpj = 4, kRedSpj = 5,
  kRedRefreshed = 6, kRedOverflow = 7, kRedTotInter = 8, kRedTotInterSpj = 9,
  kRedTotRefreshed = 10, kRedTotOverflow = 11, kRedCount = 16
};

// A device buffer that only grows.
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t cap = 0;
};

// Longest-first order of the last items of each XCD's stretch of the force
// launch, and the stretches (item indices b[0..8]) it was made for.
struct TailOrder {
  DBuf<uint32_t> order;
  int64_t b[9] = {};
  bool valid = false;
};

struct TimerRec {
  int phase;
  hipEvent_t a, b;
};

}  // namespace nb

struct nb_ctx {
  nb_config cfg;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // A construction step's moment pass runs on `side`, beside the walk that
  // follows it on `stream` (the walk needs the cells and group boxes, not
  // the moments); mom_done marks its end, and join_moments makes `stream`
  // wait for it before anything reads the moments.
  hipStream_t side = nullptr;
  hipEvent_t mom_fork = nullptr, mom_done = nullptr;
  bool mom_pending = false;
  int device = 0;
  std::string err;

  // sizes of the current particle set, tree and lists
  int64_t n = 0, n_cell = 0, n_groups = 0, n_wi = 0, n_leaves = 0;
  // independent systems: particles [sys_off[s], sys_off[s + 1]) form
  // system s (one system unless nb_set_systems says otherwise)
  int64_t n_sys = 1;
  std::vector<int64_t> h_sys_off;
  std::vector<int4> h_bbox_chunks;  // system, begin, end, first partial
  int64_t n_epj = 0, n_spj = 0, n_inter = 0;
  // token slots per group of the one-pass walk (0: count pass first); set
  // from the largest token count of the previous construction
  uint32_t tok_slab = 0;
  int64_t force_evals = 0, total_inter = 0;
  int64_t n_inter_spj = 0, total_inter_spj = 0;  // superparticle share
  int32_t k = 0;
  // internal cells per level and where each level starts in lvl_cells;
  // index kLevels holds the leaves
  int64_t lvl_count[nb::kLevels + 1] = {0};
  int64_t lvl_off[nb::kLevels + 1] = {0};

  // state machine
  bool have_particles = false;
  bool tree_valid = false;       // cells/groups exist for the particle order
  bool positions_fresh = false;  // positions unchanged since the tree build
  bool lists_valid = false;      // lists match the tree
  bool lists_reusable = false;   // built with NB_MAKE_LIST_FOR_REUSE
  bool forces_valid = false;

  // particles, internal order (double-buffered for the reorder)
  nb::DBuf<double4> pos, pos2;  // x, y, z, m
  nb::DBuf<double> vx, vy, vz, vx2, vy2, vz2;
  nb::DBuf<uint32_t> orig, orig2;  // original index per internal slot
  nb::DBuf<float4> acc;            // ax, ay, az, pot (G applied)
  nb::DBuf<float4> jcopy;          // copied lists (NB_FLAG_COPIED_LISTS)

  // keys and sort
  nb::DBuf<uint64_t> key, key2;
  nb::DBuf<uint32_t> val, val2;
  nb::DBuf<uint32_t> hist;   // 256 x blocks
  nb::DBuf<uint32_t> dtot;   // 256 digit totals
  nb::DBuf<nb::Root> root;        // one per system
  nb::DBuf<double> bbox_part;
  nb::DBuf<int4> bbox_chunks;     // bbox work: {system, begin, end, 0}
  nb::DBuf<uint32_t> bbox_first;  // per system: first chunk, n_sys + 1
  nb::DBuf<uint32_t> seg;         // system of each slot
  nb::DBuf<uint32_t> sys_off;     // n_sys + 1 slot offsets
  nb::DBuf<uint32_t> croot;       // n_sys + 1: first cell of each system

  // link
  nb::DBuf<uint8_t> lam, lmin;
  nb::DBuf<uint32_t> cstart;  // cells starting at each particle -> scanned

  // cells (DFS pre-order)
  nb::DBuf<nb::CellRec> c_rec;
  nb::DBuf<uint4> c_wrec;    // 16-byte walk records, same ids
  nb::DBuf<float4> c_mom;    // COM offset from the centre (FP32), mass
  nb::DBuf<float4> c_quad;   // 2 per cell: xx yy zz xy | xz yz 0 0
  nb::DBuf<double4> c_pm;    // absolute COM (FP64) and mass: SPJ record
  nb::DBuf<uint32_t> lvl_cells;  // cell ids grouped by level, leaves last
  nb::DBuf<uint32_t> bucket;     // per-block level histograms, scanned
  nb::DBuf<uint32_t> lvl_stage;  // level starts and group count, for the host
  // moments in two launches: blocks (maximal subtrees of at most
  // kMomBlock cells, by root id) and the cells above them (top cells, by
  // level; tlo = where each level starts) with their child table (8 ids per
  // top cell, by octant); the scanned flags that made them; their counts
  nb::DBuf<uint32_t> mp_bflag, mp_tflag, mp_blocks, mp_top, mp_tlo, mp_ctab;
  // the terms each block's root adds to its parent's sums, by child-table
  // slot (monopole moments; written by the block launch for the top launch)
  nb::DBuf<float4> mp_slot;
  int64_t mp_nblk = 0, mp_ntop = 0, mp_slot_cap = 0;

  // groups
  nb::DBuf<uint32_t> gflag;  // n_cell + 1, scanned
  nb::DBuf<uint32_t> g_cell, g_begin, g_count;
  nb::DBuf<double4> g_lo, g_hi;  // tight box of the members (w unused)
  nb::DBuf<uint32_t> g_chunks;  // n_groups + 1, scanned
  nb::DBuf<uint4> wi;           // force work items: group, first, count
  // force launch plan: XCD x takes work items [xcd_b[x], xcd_b[x + 1]),
  // split where the estimated cost of the items is balanced
  nb::DBuf<uint32_t> g_cost;     // n_groups: estimated cost of each group
  nb::DBuf<uint64_t> g_cost_off; // n_groups + 1, scanned
  nb::DBuf<uint64_t> xcd_plan;   // 9 item indices
  int64_t xcd_b[9] = {};
  int64_t nbr_b[9] = {};         // the same for the SPH density launch
  // longest-first order of the last items of each XCD's stretch
  nb::TailOrder tail;
  nb::DBuf<unsigned int> queue;  // per-XCD counters of the persistent launch

  // short-range neighbour lists (nb_neighbour_lists): per group the
  // particle-slot candidates within the search radius nbr_h, and the SPH
  // densities computed on them
  bool nbr_valid = false, rho_valid = false;
  double nbr_h = 0.0;
  int64_t n_nbr = 0;
  nb::DBuf<uint32_t> nb_cnt, nb_tcnt, nb_ids;
  nb::DBuf<uint32_t> nb_tcnt_a;  // tokens of the first half of each walk
  nb::DBuf<uint64_t> nb_off, nb_toff;
  nb::DBuf<float> rho;

  // lists
  nb::DBuf<uint32_t> cnt_e, cnt_s, cnt_t;
  nb::DBuf<uint32_t> cnt_tl;  // tokens of each lane of a split walk
                              // (nb::kSplitLanes per group)
  bool walk_split = false;    // the last walk ran kSplitLanes lanes per group
  nb::DBuf<uint64_t> epj_off, spj_off, tok_off;
  nb::DBuf<uint32_t> epj, spj, tok;  // tok: walk tokens per group
  nb::DBuf<unsigned> lflag;          // check of uploaded lists

  // scan / reduction scratch
  nb::DBuf<uint64_t> scan_tmp;
  nb::DBuf<uint64_t> red;  // small reductions and counters (kRed*)
  const uint64_t* red_zeroed = nullptr;  // red's allocation whose counters
                                         // were set to zero
  void* h_small = nullptr; // pinned host staging (4 KiB)

  // per-group list refresh (NB_FLAG_REFRESH)
  bool learn = false;        // refresh mode of the current configuration
  bool in_build = false;     // inside a construction step
  bool shift_fresh = false;  // centres of mass match the positions
  nb::DBuf<double4> c_com, c_com0;  // FP64 centre of mass (w = mass): now,
                                    // and at construction
  nb::DBuf<double4> c_bmin, c_bmax;  // box of each cell's particles now
  nb::DBuf<double4> c_shift;        // com - com0, w = side in the test
  nb::DBuf<double4> c_ctr;          // geo + shift, w = (side/theta)^2
  nb::DBuf<double4> g_clo, g_chi;   // current tight boxes
  nb::DBuf<double4> g_tau0;         // cell shift when the list was walked
  nb::DBuf<double> g_sa, g_so;      // opening-test slacks of that walk
  nb::DBuf<uint32_t> g_age;         // reuse steps since that walk
  nb::DBuf<uint32_t> pick, pickpos, sel;  // refresh selection
  nb::DBuf<uint32_t> ne2, ns2;              // list slot capacities
  // a refresh walk's output per selection slot: counts, walk state, and
  // whether the new list fits the group's slot
  nb::DBuf<uint32_t> sel_e, sel_s, sel_t;
  nb::DBuf<double> sel_sa, sel_so;
  nb::DBuf<double4> sel_tau0;
  nb::DBuf<uint8_t> sel_ok;
  // larger list slots, when an explicit refresh outgrows them
  nb::DBuf<uint64_t> epj_off2, spj_off2;
  nb::DBuf<uint32_t> epj2, spj2;
  // refresh mode: each group's lists sit in a slot with room to grow (the
  // offsets are the slots' starts, cnt_e / cnt_s the lengths); the totals of
  // the slots
  int64_t cap_e = 0, cap_s = 0;
  // refresh mode: room for the tokens of each lane of a refresh walk
  // (kSplitLanes per group, by group id: CSR offsets into tok, twice the
  // lane's tokens at construction plus kLaneSpare, 16-aligned), and its
  // total
  nb::DBuf<uint32_t> lane_cap;
  nb::DBuf<uint64_t> lane_off, lane_off2;
  int64_t lane_total = 0;
  int64_t host_refreshed = 0;  // groups refreshed by nb_refresh_lists
  nb::DBuf<float> feat, prob;       // predictor inputs [G x 12], outputs
  nb::DBuf<uint8_t> stale;          // labels of the last stale walk
  // perceptron: weights, Adam moments, gradient (+ loss), scratch
  nb::DBuf<float> mlp_w, mlp_m, mlp_v, mlp_g;
  nb::DBuf<float> mlp_act, mlp_dz, mlp_lossp, mlp_part, mlp_x, mlp_y;
  int64_t mlp_t = 0;

  // captured reuse step (NB_FLAG_GRAPH)
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  double graph_dtk = 0.0, graph_dtd = 0.0;
  int graph_mode = -1;

  // timing
  std::vector<nb::TimerRec> timers;
  std::vector<hipEvent_t> ev_pool;
  double ph_ms[NB_PH_COUNT] = {0};
  int64_t ph_calls[NB_PH_COUNT] = {0};
};

namespace nb {

// ---- error helpers (nb_api.hip) ----
int set_err(nb_ctx* c, int code, const char* fmt, ...);
int hip_check(nb_ctx* c, hipError_t e, const char* what);

template <class T>
int reserve(nb_ctx* c, DBuf<T>& b, size_t n) {
  if (n <= b.cap) return NB_OK;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    if (e != hipSuccess) return hip_check(c, e, "hipFree");
  }
  size_t want = n + n / 4 + 64;
  void* p = nullptr;
  if (hipMalloc(&p, want * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return set_err(c, NB_ERR_OOM, "device allocation of %zu bytes failed",
                   want * sizeof(T));
  }
  b.p = static_cast<T*>(p);
  b.cap = want;
  return NB_OK;
}

template <class T>
void release(DBuf<T>& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

// timers and host synchronisation (nb_api.hip)
void timer_begin(nb_ctx* c, int phase, hipEvent_t* a);
void timer_end(nb_ctx* c, int phase, hipEvent_t a);
struct Timed {
  nb_ctx* c;
  int ph;
  hipEvent_t a;
  Timed(nb_ctx* c_, int ph_) : c(c_), ph(ph_) { timer_begin(c, ph, &a); }
  ~Timed() { timer_end(c, ph, a); }
};
int stage_d2h(nb_ctx* c, size_t off, const void* src, size_t bytes);
int sync_stream(nb_ctx* c);
void join_moments(nb_ctx* c);  // stream waits for a side-stream moment pass
void drop_graph(nb_ctx* c);  // a captured step refers to the list buffers

// ---- stage launchers; all enqueue on c->stream and return a status ----
// nb_scan.hip
int scan_u32(nb_ctx* c, const uint32_t* in, uint32_t* out, int64_t n);
int scan_u32_to_u64(nb_ctx* c, const uint32_t* in, uint64_t* out, int64_t n);
int radix_sort(nb_ctx* c, int64_t n);  // key/val -> key/val (sorted)
// nb_tree.hip
int launch_root(nb_ctx* c);
int launch_keys(nb_ctx* c);
int launch_reorder(nb_ctx* c);
int launch_link_count(nb_ctx* c);
int launch_link_fill(nb_ctx* c);
int launch_level_lists(nb_ctx* c);  // enqueues; no host sync
// blocks and top cells of the two-launch moments, after the level lists;
// stages their counts after the level starts and group count
int launch_mom_plan(nb_ctx* c);
int launch_moments(nb_ctx* c);
int launch_group_flags(nb_ctx* c);
int launch_sys_roots(nb_ctx* c);
int launch_seg_fill(nb_ctx* c);
int launch_group_fill(nb_ctx* c);
int launch_group_box(nb_ctx* c, double4* lo, double4* hi);
// nb_walk.hip
int launch_walk(nb_ctx* c, bool fill, uint32_t slab = 0);
int launch_walk_sel(nb_ctx* c, bool fill, int64_t n_walk, const double4* lo,
                    const double4* hi, const uint64_t* epj_off,
                    const uint64_t* spj_off, uint32_t* epj, uint32_t* spj,
                    uint32_t slab = 0);
// Refresh walk over up to n_max selected groups (count *o.n_dev on the
// device), kSplitLanes lanes per group, one pass: each lane's tokens into
// its group's lane range (lane_off), its count into cnt_tl (per slot).
int launch_walk_refresh(nb_ctx* c, int64_t n_max, const uint32_t* sel,
                        const double4* lo, const double4* hi,
                        const WalkOut& o);
// Expand of a refresh walk's slots t with ok[t] into their groups' lists.
int launch_expand_sel(nb_ctx* c, int64_t n_max, const uint32_t* sel,
                      const uint32_t* n_dev, const uint8_t* ok);
// Room of each refresh-walk lane from the construction walk's lane counts
// (lane_cap, then its scan into lane_off; total at lane_off[G S]).
int launch_lane_room(nb_ctx* c);
// per-force-call device counters (refresh mode); refresh_step adds the
// call's refreshed groups, otherwise they are cleared
int launch_accum(nb_ctx* c, bool refresh_step);
int launch_expand_slab(nb_ctx* c, uint32_t slab);
int walk_tile(int64_t n_walk);  // lanes per tile of the walk (1: split)
bool split_walk(const nb_ctx* c, int64_t n_walk);  // kSplitLanes slabs per group
int launch_list_stats(nb_ctx* c);
// short-range walk: count pass (nb_cnt, nb_tcnt and their scans) and, with
// the totals known, the fill pass and expand into nb_ids
int launch_nbr_count(nb_ctx* c, double h);
int launch_nbr_fill(nb_ctx* c, double h);
// SPH density on the neighbour lists into c->rho
int launch_density(nb_ctx* c, double h);
int launch_interactions(nb_ctx* c, const uint32_t* ne, const uint32_t* ns);
int launch_check_lists(nb_ctx* c, unsigned* flag);  // uploaded lists
// nb_learn.hip
int learn_reserve_cells(nb_ctx* c);
int learn_reserve_groups(nb_ctx* c);
int launch_com(nb_ctx* c);
int learn_after_groups(nb_ctx* c);
int launch_age_inc(nb_ctx* c);
int launch_features(nb_ctx* c);
int launch_stale(nb_ctx* c, double tau);
int mlp_ensure(nb_ctx* c);
// device address of the static scratch of nb_mlp_grad_static, once per GPU
int static_scratch_init(nb_ctx* c);
int mlp_forward(nb_ctx* c, int64_t n, const float* x, float* p);
int mlp_grad(nb_ctx* c, int64_t n, const float* x, const float* y, float pw);
int mlp_adam(nb_ctx* c, const float* g, float lr, float b1, float b2,
             float eps);
int refresh_selected(nb_ctx* c);
int refresh_host_sel(nb_ctx* c, int64_t n_sel, const int64_t* sel);
int refresh_predicted(nb_ctx* c);
int refresh_checked(nb_ctx* c);
int labels_to_float(nb_ctx* c, float* out);
// nb_force.hip
int launch_force(nb_ctx* c);
// device plan of the force (or SPH density) launch, read back with the
// lists' totals into xcd_b (nbr_b)
int launch_xcd_plan(nb_ctx* c, bool neighbours);
int launch_tail_order(nb_ctx* c);  // after the plan is read back
// nb_step.hip
int launch_kick_drift(nb_ctx* c, double dt_kick, double dt_drift);
int launch_pack(nb_ctx* c, const double* x, const double* y, const double* z,
                const double* m);
int fill_u32(nb_ctx* c, uint32_t* p, int64_t n, uint32_t v);

inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace nb
