// nb_api.hip -- the C ABI of libnbody_hip.so: context, memory, the
// construction / reuse state machine of the paper's reuse modes (section 4.2
// and section 5), host synchronisation points and readback.
//
// A construction step synchronises with the host three times, to size
// buffers: after the cell count, after the group count and level histogram,
// and after the list lengths.  A reuse step does not synchronise.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "nb_internal.h"

namespace nb {

int set_err(nb_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

int hip_check(nb_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return NB_OK;
  return set_err(c, NB_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

static hipEvent_t take_event(nb_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

static void resolve_timers(nb_ctx* c) {
  for (auto& t : c->timers) {
    float ms = 0.f;
    if (hipEventSynchronize(t.b) == hipSuccess &&
        hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      c->ph_ms[t.phase] += ms;
      c->ph_calls[t.phase] += 1;
    } else {
      (void)hipGetLastError();
    }
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->timers.clear();
}

void timer_begin(nb_ctx* c, int phase, hipEvent_t* a) {
  (void)phase;
  *a = nullptr;
  if (!(c->cfg.flags & 1)) return;
  hipEvent_t e = take_event(c);
  if (e && hipEventRecord(e, c->stream) == hipSuccess) {
    *a = e;
  } else if (e) {
    (void)hipGetLastError();
    c->ev_pool.push_back(e);
  }
}

void timer_end(nb_ctx* c, int phase, hipEvent_t a) {
  if (!a) return;
  hipEvent_t b = take_event(c);
  if (!b || hipEventRecord(b, c->stream) != hipSuccess) {
    (void)hipGetLastError();
    c->ev_pool.push_back(a);
    if (b) c->ev_pool.push_back(b);
    return;
  }
  c->timers.push_back(TimerRec{phase, a, b});
  if (c->timers.size() > 4096) resolve_timers(c);
}

static int check_cfg(nb_ctx* c, const nb_config* cfg) {
  if (!cfg) return set_err(c, NB_ERR_INPUT, "config is NULL");
  if (!(cfg->theta >= 0.0) || !std::isfinite(cfg->theta))
    return set_err(c, NB_ERR_INPUT, "theta must be finite and >= 0");
  if (!(cfg->eps > 0.0) || !std::isfinite(cfg->eps))
    return set_err(c, NB_ERR_INPUT, "eps must be finite and > 0");
  if (!std::isfinite(cfg->G) || !std::isfinite(cfg->ext_mass))
    return set_err(c, NB_ERR_INPUT, "G and ext_mass must be finite");
  if (cfg->n_leaf < 1 || cfg->n_leaf > 64)
    return set_err(c, NB_ERR_INPUT, "n_leaf must be in 1..64");
  if (cfg->n_grp < 1 || cfg->n_grp > 65536)
    return set_err(c, NB_ERR_INPUT, "n_grp must be in 1..65536");
  if (cfg->order != 1 && cfg->order != 2)
    return set_err(c, NB_ERR_INPUT, "order must be 1 or 2");
  if ((cfg->flags & NB_FLAG_COPIED_LISTS) &&
      (cfg->order != 1 || (cfg->flags & (NB_FLAG_REFRESH | NB_FLAG_PERSISTENT))))
    return set_err(c, NB_ERR_INPUT,
                   "copied lists need order 1, no refresh mode and no "
                   "persistent launch");
  if (!(cfg->tile_j == 0 || cfg->tile_j == 64 || cfg->tile_j == 128 ||
        cfg->tile_j == 192 || cfg->tile_j == 256))
    return set_err(c, NB_ERR_INPUT, "tile_j must be 0, 64, 128, 192 or 256");
  if (!(cfg->waves_per_simd == 0 || cfg->waves_per_simd == 4 ||
        cfg->waves_per_simd == 6 || cfg->waves_per_simd == 8))
    return set_err(c, NB_ERR_INPUT, "waves_per_simd must be 0, 4, 6 or 8");
  if (cfg->flags & NB_FLAG_REFRESH) {
    if (cfg->k_max < 1 || cfg->k_max > 65535)
      return set_err(c, NB_ERR_INPUT, "k_max must be in 1..65535");
    if (!(cfg->p_star >= 0.0 && cfg->p_star <= 1.0))
      return set_err(c, NB_ERR_INPUT, "p_star must be in [0, 1]");
    if (!(cfg->tau >= 0.0) || !std::isfinite(cfg->tau))
      return set_err(c, NB_ERR_INPUT, "tau must be finite and >= 0");
  }
  return NB_OK;
}

// Copy `bytes` from device to the pinned staging buffer at `off` (async).
int stage_d2h(nb_ctx* c, size_t off, const void* src, size_t bytes) {
  return hip_check(c,
                   hipMemcpyAsync(static_cast<char*>(c->h_small) + off, src,
                                  bytes, hipMemcpyDeviceToHost, c->stream),
                   "staging copy");
}

void join_moments(nb_ctx* c) {
  if (!c->mom_pending) return;
  c->mom_pending = false;
  if (hipStreamWaitEvent(c->stream, c->mom_done, 0) != hipSuccess) {
    // ordering by a full wait instead
    (void)hipGetLastError();
    (void)hipStreamSynchronize(c->side);
  }
}

int sync_stream(nb_ctx* c) {
  return hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
}

static int sync(nb_ctx* c) { return sync_stream(c); }

void drop_graph(nb_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
}

static int build_tree(nb_ctx* c) {
  if (!c->have_particles)
    return set_err(c, NB_ERR_STATE, "no particles set");
  int rc;
  drop_graph(c);
  c->tree_valid = c->positions_fresh = false;
  c->lists_valid = c->lists_reusable = c->forces_valid = false;
  c->nbr_valid = c->rho_valid = false;
  {
    Timed t(c, NB_PH_ROOT);
    if ((rc = launch_root(c))) return rc;
  }
  {
    Timed t(c, NB_PH_KEYS);
    if ((rc = launch_keys(c))) return rc;
  }
  {
    Timed t(c, NB_PH_SORT);
    if ((rc = radix_sort(c, c->n))) return rc;
  }
  {
    Timed t(c, NB_PH_REORDER);
    if ((rc = launch_reorder(c))) return rc;
  }
  {
    Timed t(c, NB_PH_LINK);
    if ((rc = launch_link_count(c))) return rc;
  }
  // sync 1: number of cells, root exponent, finiteness of the input
  if ((rc = stage_d2h(c, 0, c->cstart.p + c->n, sizeof(uint32_t)))) return rc;
  if ((rc = stage_d2h(c, 8, &c->root.p->k, 2 * sizeof(int32_t)))) return rc;
  if ((rc = sync(c))) return rc;
  {
    const uint32_t* h = static_cast<const uint32_t*>(c->h_small);
    const int32_t* hk = reinterpret_cast<const int32_t*>(
        static_cast<const char*>(c->h_small) + 8);
    if (hk[1]) return set_err(c, NB_ERR_INPUT, "non-finite particle position");
    c->k = hk[0];
    c->n_cell = h[0];
  }
  if (c->n_cell < 1 || c->n_cell >= (int64_t)kNone)
    return set_err(c, NB_ERR_HIP, "cell count out of range (%lld)",
                   (long long)c->n_cell);
  {
    Timed t(c, NB_PH_LINK);
    if ((rc = launch_link_fill(c))) return rc;
  }
  {
    Timed t(c, NB_PH_GROUPS);
    if ((rc = launch_group_flags(c))) return rc;
    if ((rc = launch_level_lists(c))) return rc;
    if ((rc = launch_mom_plan(c))) return rc;
  }
  // sync 2: where each level starts in the level lists (the leaves are
  // bucket kLevels), the group count, and the block and top-cell counts of
  // the moment pass
  if ((rc = stage_d2h(c, 0, c->lvl_stage.p, (kLevels + 4) * sizeof(uint32_t))))
    return rc;
  if ((rc = sync(c))) return rc;
  {
    const uint32_t* h = static_cast<const uint32_t*>(c->h_small);
    for (int b = 0; b <= kLevels; ++b) {
      c->lvl_off[b] = h[b];
      const int64_t next = b < kLevels ? (int64_t)h[b + 1] : c->n_cell;
      c->lvl_count[b] = next - (int64_t)h[b];
      if (c->lvl_count[b] < 0)
        return set_err(c, NB_ERR_HIP, "inconsistent level histogram");
    }
    c->n_leaves = c->lvl_count[kLevels];
    c->n_groups = h[kLevels + 1];
    c->mp_nblk = h[kLevels + 2];
    c->mp_ntop = h[kLevels + 3];
    if (c->n_groups < 1 || h[0] != 0)
      return set_err(c, NB_ERR_HIP, "inconsistent tree (%lld groups)",
                     (long long)c->n_groups);
  }
  {
    // The moment pass goes to the side stream and runs beside the group
    // boxes and the walk; the force launch and every reader of the moments
    // join it first.  In refresh mode the walk reads the centres this pass
    // sets, so there it stays on the stream.
    const bool side = !c->learn && c->side;
    hipStream_t main = c->stream;
    if (side) {
      if ((rc = hip_check(c, hipEventRecord(c->mom_fork, main),
                          "moment fork")) ||
          (rc = hip_check(c, hipStreamWaitEvent(c->side, c->mom_fork, 0),
                          "moment fork wait")))
        return rc;
      c->stream = c->side;
    }
    {
      Timed t(c, NB_PH_MOMENTS);
      c->in_build = true;
      rc = launch_moments(c);
      c->in_build = false;
    }
    if (side) {
      const hipError_t e = hipEventRecord(c->mom_done, c->side);
      c->stream = main;
      c->mom_pending = true;
      if (!rc) rc = hip_check(c, e, "moment join event");
    }
    if (rc) return rc;
  }
  {
    Timed t(c, NB_PH_GROUPS);
    if ((rc = launch_group_fill(c))) return rc;
    if (c->learn && (rc = learn_after_groups(c))) return rc;
  }
  c->tree_valid = c->positions_fresh = true;
  c->shift_fresh = c->learn;
  return NB_OK;
}

static int make_lists(nb_ctx* c, nb_mode mode) {
  if (mode == NB_REUSE_LIST || mode == NB_REUSE_REFRESH ||
      mode == NB_REUSE_CHECK)
    return c->lists_reusable ? NB_OK
                             : set_err(c, NB_ERR_STATE, "no reusable lists");
  if (mode != NB_MAKE_LIST && mode != NB_MAKE_LIST_FOR_REUSE)
    return set_err(c, NB_ERR_INPUT, "bad mode %d", (int)mode);
  if (!c->tree_valid || !c->positions_fresh)
    return set_err(c, NB_ERR_STATE, "lists need a tree of the current positions");
  int rc;
  c->lists_valid = c->lists_reusable = false;
  c->tail.valid = false;
  // one pass (counts and tokens into per-group slabs sized from the last
  // construction) when the slabs fit in a bounded buffer; otherwise, or when
  // a group overflows its slab, a count pass and an exact fill pass
  const uint32_t slab = c->tok_slab;
  const uint64_t slabs = split_walk(c, c->n_groups) ? kSplitLanes : 1u;
  const bool one_pass = slab > 0 &&
                        (uint64_t)c->n_groups * slabs * slab < (1ull << 32);
  if (one_pass) {
    Timed t(c, NB_PH_WALK);
    if ((rc = reserve(c, c->tok, (size_t)(c->n_groups * slabs * slab))))
      return rc;
    if ((rc = launch_walk(c, true, slab))) return rc;
    if ((rc = launch_list_stats(c))) return rc;
  } else {
    Timed t(c, NB_PH_WALK);
    if ((rc = launch_walk(c, false))) return rc;
    if ((rc = launch_list_stats(c))) return rc;
  }
  {
    Timed t(c, NB_PH_WALK);
    if ((rc = launch_xcd_plan(c, false))) return rc;
  }
  // sync 3: list totals, interaction count, force work items, largest
  // token count, force launch plan
  if ((rc = stage_d2h(c, 64, c->xcd_plan.p, 9 * 8))) return rc;
  if ((rc = stage_d2h(c, 0, c->epj_off.p + c->n_groups, 8))) return rc;
  if ((rc = stage_d2h(c, 8, c->spj_off.p + c->n_groups, 8))) return rc;
  if ((rc = stage_d2h(c, 16, c->red.p, 16))) return rc;
  if ((rc = stage_d2h(c, 32, c->tok_off.p + c->n_groups, 8))) return rc;
  if ((rc = stage_d2h(c, 40, c->g_chunks.p + c->n_groups, 4))) return rc;
  if ((rc = stage_d2h(c, 48, c->red.p + 2, 8))) return rc;
  if ((rc = stage_d2h(c, 144, c->red.p + kRedEpj, 16))) return rc;
  if (c->learn && (rc = stage_d2h(c, 160, c->lane_off.p +
                                               kSplitLanes * c->n_groups, 8)))
    return rc;
  if ((rc = sync(c))) return rc;
  int64_t n_tok, max_tok;
  {
    const uint64_t* h = static_cast<const uint64_t*>(c->h_small);
    // list entries; in refresh mode the offsets' totals are the slots'
    c->cap_e = (int64_t)h[0];
    c->cap_s = (int64_t)h[1];
    c->n_epj = (int64_t)h[18];
    c->n_spj = (int64_t)h[19];
    c->n_inter = (int64_t)h[2];
    max_tok = (int64_t)h[3];
    n_tok = (int64_t)h[4];
    c->n_inter_spj = (int64_t)h[6];
    c->n_wi = static_cast<const uint32_t*>(c->h_small)[10];
    for (int x = 0; x <= 8; ++x) c->xcd_b[x] = (int64_t)h[8 + x];
    if (c->learn) c->lane_total = (int64_t)h[20];
  }
  // slab for the next construction: 1.25 x the largest token count of one
  // slab (a group's, or one lane's of a split walk), 16-aligned
  c->tok_slab = (uint32_t)std::min<int64_t>(
      (max_tok + max_tok / 4 + 16 + 15) / 16 * 16, 1 << 24);
  {
    Timed t(c, NB_PH_WALK);
    if ((rc = launch_tail_order(c))) return rc;
  }
  if ((rc = reserve(c, c->epj, (size_t)c->cap_e + 1))) return rc;
  if ((rc = reserve(c, c->spj, (size_t)c->cap_s + 1))) return rc;
  if (one_pass && max_tok <= (int64_t)slab) {
    Timed t(c, NB_PH_WALK);
    if ((rc = launch_expand_slab(c, slab))) return rc;
  } else {
    if ((rc = reserve(c, c->tok, (size_t)n_tok + 1))) return rc;
    Timed t(c, NB_PH_WALK);
    if ((rc = launch_walk(c, true))) return rc;
  }
  // the refresh walks' token room, sized here, after the construction's
  // own tokens have been expanded, so that a refresh step allocates nothing
  if (c->learn && (rc = reserve(c, c->tok, (size_t)c->lane_total + 1)))
    return rc;
  c->lists_valid = true;
  c->lists_reusable = mode == NB_MAKE_LIST_FOR_REUSE;
  return NB_OK;
}

// The side stream of the moment pass and its two events.
static void release_side(nb_ctx* c) {
  if (c->mom_fork) (void)hipEventDestroy(c->mom_fork);
  if (c->mom_done) (void)hipEventDestroy(c->mom_done);
  if (c->side) (void)hipStreamDestroy(c->side);
  c->mom_fork = c->mom_done = nullptr;
  c->side = nullptr;
}

}  // namespace nb

using namespace nb;

extern "C" {

const char* nb_version(void) { return "nbody_hip 0.1 (gfx950)"; }

const char* nb_last_error(const nb_ctx* ctx) {
  return ctx ? ctx->err.c_str() : "no context";
}

int nb_create(const nb_config* cfg, nb_ctx** out) {
  if (!out) return NB_ERR_INPUT;
  *out = nullptr;
  int rc = check_cfg(nullptr, cfg);
  if (rc) return rc;
  nb_ctx* c = new (std::nothrow) nb_ctx();
  if (!c) return NB_ERR_OOM;
  c->cfg = *cfg;
  c->learn = (cfg->flags & NB_FLAG_REFRESH) != 0;
  if (hipGetDevice(&c->device) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return NB_ERR_HIP;
  }
  if (cfg->stream) {
    c->stream = static_cast<hipStream_t>(cfg->stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) !=
        hipSuccess) {
      (void)hipGetLastError();
      delete c;
      return NB_ERR_HIP;
    }
    c->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) !=
          hipSuccess ||
      hipEventCreateWithFlags(&c->mom_fork, hipEventDisableTiming) !=
          hipSuccess ||
      hipEventCreateWithFlags(&c->mom_done, hipEventDisableTiming) !=
          hipSuccess) {
    (void)hipGetLastError();
    release_side(c);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return NB_ERR_HIP;
  }
  if (static_scratch_init(c)) {
    release_side(c);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return NB_ERR_HIP;
  }
  if (hipHostMalloc(&c->h_small, 4096, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    release_side(c);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return NB_ERR_OOM;
  }
  *out = c;
  return NB_OK;
}

void nb_destroy(nb_ctx* c) {
  if (!c) return;
  if (c->side) (void)hipStreamSynchronize(c->side);
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  for (auto& t : c->timers) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  release(c->pos); release(c->pos2);
  release(c->vx); release(c->vy); release(c->vz);
  release(c->vx2); release(c->vy2); release(c->vz2);
  release(c->orig); release(c->orig2); release(c->acc);
  release(c->jcopy);
  release(c->key); release(c->key2); release(c->val); release(c->val2);
  release(c->hist); release(c->dtot); release(c->root); release(c->bbox_part);
  release(c->bbox_chunks); release(c->bbox_first); release(c->seg);
  release(c->sys_off); release(c->croot);
  release(c->lam); release(c->lmin); release(c->cstart);
  release(c->c_rec); release(c->c_wrec);
  release(c->c_mom); release(c->c_quad); release(c->c_pm);
  release(c->lvl_cells); release(c->bucket);
  release(c->mp_bflag); release(c->mp_tflag); release(c->mp_blocks);
  release(c->mp_top); release(c->mp_tlo); release(c->mp_ctab);
  release(c->mp_slot);
  release(c->gflag); release(c->g_cell); release(c->g_begin);
  release(c->g_count); release(c->g_lo); release(c->g_hi);
  release(c->g_chunks); release(c->wi); release(c->queue);
  release(c->g_cost); release(c->g_cost_off); release(c->xcd_plan);
  release(c->cnt_tl); release(c->tail.order);
  release(c->nb_cnt); release(c->nb_tcnt); release(c->nb_ids);
  release(c->nb_tcnt_a);
  release(c->nb_off); release(c->nb_toff); release(c->rho);
  release(c->cnt_e); release(c->cnt_s); release(c->cnt_t);
  release(c->epj_off); release(c->spj_off); release(c->tok_off);
  release(c->epj); release(c->spj); release(c->tok); release(c->lflag);
  release(c->scan_tmp); release(c->red); release(c->lvl_stage);
  release(c->c_com); release(c->c_com0); release(c->c_shift); release(c->c_ctr);
  release(c->c_bmin); release(c->c_bmax);
  release(c->g_clo); release(c->g_chi); release(c->g_tau0);
  release(c->g_sa); release(c->g_so); release(c->g_age);
  release(c->pick); release(c->pickpos); release(c->sel);
  release(c->ne2); release(c->ns2); release(c->sel_e); release(c->sel_s);
  release(c->sel_t); release(c->sel_sa); release(c->sel_so);
  release(c->sel_tau0); release(c->sel_ok); release(c->feat); release(c->prob);
  release(c->epj_off2); release(c->spj_off2); release(c->epj2);
  release(c->spj2);
  release(c->lane_cap); release(c->lane_off); release(c->lane_off2);
  release(c->stale);
  release(c->mlp_w); release(c->mlp_m); release(c->mlp_v); release(c->mlp_g);
  release(c->mlp_act); release(c->mlp_dz); release(c->mlp_lossp);
  release(c->mlp_part); release(c->mlp_x); release(c->mlp_y);
  if (c->h_small) (void)hipHostFree(c->h_small);
  release_side(c);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

int nb_set_config(nb_ctx* c, const nb_config* cfg) {
  if (!c) return NB_ERR_INPUT;
  int rc = check_cfg(c, cfg);
  if (rc) return rc;
  void* keep_stream = c->cfg.stream;
  c->cfg = *cfg;
  c->cfg.stream = keep_stream;  // the stream is fixed at creation
  c->learn = (cfg->flags & NB_FLAG_REFRESH) != 0;
  c->shift_fresh = false;
  drop_graph(c);
  c->tree_valid = c->positions_fresh = false;
  c->lists_valid = c->lists_reusable = false;
  c->tail.valid = false;
  c->nbr_valid = c->rho_valid = false;
  return NB_OK;
}

int nb_set_particles(nb_ctx* c, int64_t n, const double* x, const double* y,
                     const double* z, const double* vx, const double* vy,
                     const double* vz, const double* m, int on_device) {
  if (!c) return NB_ERR_INPUT;
  if (n < 1 || n >= 0x7FFFFFFFLL)
    return set_err(c, NB_ERR_INPUT, "n out of range (%lld)", (long long)n);
  if (!x || !y || !z || !vx || !vy || !vz || !m)
    return set_err(c, NB_ERR_INPUT, "NULL particle array");
  c->have_particles = false;
  drop_graph(c);
  c->tree_valid = c->positions_fresh = false;
  c->lists_valid = c->lists_reusable = c->forces_valid = false;
  c->nbr_valid = c->rho_valid = false;
  const size_t un = (size_t)n;
  int rc = reserve(c, c->pos, un);
  if (!rc) rc = reserve(c, c->vx, un);
  if (!rc) rc = reserve(c, c->vy, un);
  if (!rc) rc = reserve(c, c->vz, un);
  if (!rc) rc = reserve(c, c->orig, un);
  if (!rc) rc = reserve(c, c->acc, un);
  if (rc) return rc;
  c->n = n;
  const size_t bytes = un * sizeof(double);
  if (on_device) {
    rc = launch_pack(c, x, y, z, m);
    if (rc) return rc;
    rc = hip_check(c, hipMemcpyAsync(c->vx.p, vx, bytes,
                                     hipMemcpyDeviceToDevice, c->stream),
                   "vx copy");
    if (!rc) rc = hip_check(c, hipMemcpyAsync(c->vy.p, vy, bytes,
                                              hipMemcpyDeviceToDevice,
                                              c->stream), "vy copy");
    if (!rc) rc = hip_check(c, hipMemcpyAsync(c->vz.p, vz, bytes,
                                              hipMemcpyDeviceToDevice,
                                              c->stream), "vz copy");
    if (!rc) rc = sync(c);
    if (rc) return rc;
  } else {
    std::vector<double4> hp(un);
    std::vector<uint32_t> ho(un);
    for (size_t i = 0; i < un; ++i) {
      hp[i] = make_double4(x[i], y[i], z[i], m[i]);
      ho[i] = (uint32_t)i;
    }
    rc = sync(c);
    if (!rc) rc = hip_check(c, hipMemcpy(c->pos.p, hp.data(), un * sizeof(double4),
                                         hipMemcpyHostToDevice), "pos upload");
    if (!rc) rc = hip_check(c, hipMemcpy(c->orig.p, ho.data(), un * 4,
                                         hipMemcpyHostToDevice), "orig upload");
    if (!rc) rc = hip_check(c, hipMemcpy(c->vx.p, vx, bytes,
                                         hipMemcpyHostToDevice), "vx upload");
    if (!rc) rc = hip_check(c, hipMemcpy(c->vy.p, vy, bytes,
                                         hipMemcpyHostToDevice), "vy upload");
    if (!rc) rc = hip_check(c, hipMemcpy(c->vz.p, vz, bytes,
                                         hipMemcpyHostToDevice), "vz upload");
    if (rc) return rc;
  }
  c->n_sys = 1;
  c->h_sys_off.assign({0, n});
  rc = launch_seg_fill(c);
  if (rc) return rc;
  c->have_particles = true;
  return NB_OK;
}

int nb_set_systems(nb_ctx* c, int64_t n_sys, const int64_t* off) {
  if (!c) return NB_ERR_INPUT;
  if (!c->have_particles)
    return set_err(c, NB_ERR_STATE, "set the particles before the systems");
  if (n_sys < 1 || n_sys > c->n || !off)
    return set_err(c, NB_ERR_INPUT, "bad system count %lld", (long long)n_sys);
  if (off[0] != 0 || off[n_sys] != c->n)
    return set_err(c, NB_ERR_INPUT, "system offsets must run from 0 to n");
  for (int64_t s = 0; s < n_sys; ++s)
    if (off[s + 1] <= off[s])
      return set_err(c, NB_ERR_INPUT, "system %lld is empty", (long long)s);
  drop_graph(c);
  c->tree_valid = c->positions_fresh = false;
  c->lists_valid = c->lists_reusable = false;
  c->tail.valid = false;
  c->nbr_valid = c->rho_valid = false;
  c->n_sys = n_sys;
  c->h_sys_off.assign(off, off + n_sys + 1);
  return launch_seg_fill(c);
}

int nb_build_tree(nb_ctx* c) {
  if (!c) return NB_ERR_INPUT;
  const int rc = build_tree(c);
  join_moments(c);
  return rc;
}

int nb_make_lists(nb_ctx* c, nb_mode mode) {
  if (!c) return NB_ERR_INPUT;
  return make_lists(c, mode);
}

int nb_compute_forces(nb_ctx* c, nb_mode mode) {
  if (!c) return NB_ERR_INPUT;
  int rc;
  if (mode == NB_REUSE_LIST || mode == NB_REUSE_REFRESH ||
      mode == NB_REUSE_CHECK) {
    if (!c->have_particles || !c->tree_valid || !c->lists_reusable)
      return set_err(c, NB_ERR_STATE,
                     "REUSE_LIST needs lists made with MAKE_LIST_FOR_REUSE");
    if (mode != NB_REUSE_LIST && !c->learn)
      return set_err(c, NB_ERR_STATE,
                     "REUSE_REFRESH and REUSE_CHECK need NB_FLAG_REFRESH");
    if (mode == NB_REUSE_CHECK && !(c->cfg.theta > 0.0))
      return set_err(c, NB_ERR_INPUT, "REUSE_CHECK needs theta > 0");
    {
      Timed t(c, NB_PH_MOMENTS);
      if ((rc = launch_moments(c))) return rc;
    }
    if (c->learn) {
      if ((rc = launch_age_inc(c))) return rc;
      c->shift_fresh = true;
    }
    if (mode == NB_REUSE_REFRESH) {
      Timed t(c, NB_PH_REFRESH);
      if ((rc = refresh_predicted(c))) return rc;
    } else if (mode == NB_REUSE_CHECK) {
      Timed t(c, NB_PH_REFRESH);
      if ((rc = refresh_checked(c))) return rc;
    }
  } else if (mode == NB_MAKE_LIST || mode == NB_MAKE_LIST_FOR_REUSE) {
    rc = build_tree(c);
    if (!rc) rc = make_lists(c, mode);
    join_moments(c);
    if (rc) return rc;
  } else {
    return set_err(c, NB_ERR_INPUT, "bad mode %d", (int)mode);
  }
  {
    Timed t(c, NB_PH_FORCE);
    if ((rc = launch_force(c))) return rc;
  }
  // refresh mode counts on the device (the lists change without the host)
  if (c->learn &&
      (rc = launch_accum(c, mode == NB_REUSE_REFRESH || mode == NB_REUSE_CHECK)))
    return rc;
  c->forces_valid = true;
  c->force_evals += 1;
  c->total_inter += c->n_inter;
  c->total_inter_spj += c->n_inter_spj;
  return NB_OK;
}

int nb_kick_drift(nb_ctx* c, double dt_kick, double dt_drift) {
  if (!c) return NB_ERR_INPUT;
  if (!std::isfinite(dt_kick) || !std::isfinite(dt_drift))
    return set_err(c, NB_ERR_INPUT, "non-finite time step");
  if (!c->forces_valid)
    return set_err(c, NB_ERR_STATE, "kick-drift needs computed forces");
  int rc;
  {
    Timed t(c, NB_PH_KICK);
    if ((rc = launch_kick_drift(c, dt_kick, dt_drift))) return rc;
  }
  if (dt_drift != 0.0) {
    c->positions_fresh = false;
    c->shift_fresh = false;
    if (!c->lists_reusable) c->lists_valid = false;
  }
  return NB_OK;
}

// The kernels of one reuse step: kick-drift, moments of the frozen tree,
// (refresh mode) the predictor or the exact check and the refresh of the
// lists it selects, force on the kept lists.  No host synchronisation.
static int enqueue_reuse_step(nb_ctx* c, nb_mode mode, double dtk,
                              double dtd) {
  int rc = launch_kick_drift(c, dtk, dtd);
  if (!rc) rc = launch_moments(c);
  if (!rc && c->learn) rc = launch_age_inc(c);
  if (!rc && mode == NB_REUSE_REFRESH) rc = refresh_predicted(c);
  if (!rc && mode == NB_REUSE_CHECK) rc = refresh_checked(c);
  if (!rc) rc = launch_force(c);
  if (!rc && c->learn) rc = launch_accum(c, mode != NB_REUSE_LIST);
  return rc;
}

int nb_step(nb_ctx* c, nb_mode mode, double dt_kick, double dt_drift) {
  if (!c) return NB_ERR_INPUT;
  const bool graph = (c->cfg.flags & NB_FLAG_GRAPH) != 0;
  const bool reuse = mode == NB_REUSE_LIST ||
                     (c->learn && (mode == NB_REUSE_REFRESH ||
                                   mode == NB_REUSE_CHECK));
  if (!(graph && reuse)) {
    int rc = nb_kick_drift(c, dt_kick, dt_drift);
    if (!rc) rc = nb_compute_forces(c, mode);
    return rc;
  }
  if (!std::isfinite(dt_kick) || !std::isfinite(dt_drift))
    return set_err(c, NB_ERR_INPUT, "non-finite time step");
  if (!c->forces_valid)
    return set_err(c, NB_ERR_STATE, "kick-drift needs computed forces");
  if (!c->have_particles || !c->tree_valid || !c->lists_reusable)
    return set_err(c, NB_ERR_STATE,
                   "REUSE_LIST needs lists made with MAKE_LIST_FOR_REUSE");
  if (mode == NB_REUSE_CHECK && !(c->cfg.theta > 0.0))
    return set_err(c, NB_ERR_INPUT, "REUSE_CHECK needs theta > 0");
  int rc;
  if (c->graph_exec &&
      (c->graph_dtk != dt_kick || c->graph_dtd != dt_drift ||
       c->graph_mode != (int)mode))
    drop_graph(c);
  // the perceptron's weights exist before the capture (nothing is allocated
  // while the stream is captured)
  if (mode == NB_REUSE_REFRESH && (rc = mlp_ensure(c))) return rc;
  if (!c->graph_exec) {
    // buffers are already sized by the construction step, so nothing is
    // allocated while the stream is being captured
    rc = hip_check(c, hipStreamBeginCapture(c->stream,
                                            hipStreamCaptureModeRelaxed),
                   "graph capture");
    if (rc) return rc;
    const int rq = enqueue_reuse_step(c, mode, dt_kick, dt_drift);
    hipGraph_t gr = nullptr;
    const hipError_t ee = hipStreamEndCapture(c->stream, &gr);
    if (rq) {
      if (gr) (void)hipGraphDestroy(gr);
      return rq;
    }
    rc = hip_check(c, ee, "graph capture end");
    if (rc) return rc;
    c->graph = gr;
    rc = hip_check(c, hipGraphInstantiate(&c->graph_exec, gr, nullptr,
                                          nullptr, 0), "graph instantiate");
    if (rc) {
      drop_graph(c);
      return rc;
    }
    c->graph_dtk = dt_kick;
    c->graph_dtd = dt_drift;
    c->graph_mode = (int)mode;
  }
  {
    Timed t(c, NB_PH_GRAPH);
    rc = hip_check(c, hipGraphLaunch(c->graph_exec, c->stream), "graph launch");
    if (rc) return rc;
  }
  if (dt_drift != 0.0) c->positions_fresh = false;
  c->shift_fresh = c->learn;
  c->forces_valid = true;
  c->force_evals += 1;
  c->total_inter += c->n_inter;
  c->total_inter_spj += c->n_inter_spj;
  return NB_OK;
}

int nb_get_forces(nb_ctx* c, double* ax, double* ay, double* az, double* pot,
                  int internal) {
  if (!c) return NB_ERR_INPUT;
  if (!ax || !ay || !az || !pot)
    return set_err(c, NB_ERR_INPUT, "NULL output array");
  if (!c->forces_valid) return set_err(c, NB_ERR_STATE, "no forces computed");
  const size_t n = (size_t)c->n;
  std::vector<float4> a(n);
  std::vector<uint32_t> o(n);
  int rc = sync(c);
  if (!rc) rc = hip_check(c, hipMemcpy(a.data(), c->acc.p, n * sizeof(float4),
                                       hipMemcpyDeviceToHost), "acc readback");
  if (!rc) rc = hip_check(c, hipMemcpy(o.data(), c->orig.p, n * 4,
                                       hipMemcpyDeviceToHost), "orig readback");
  if (rc) return rc;
  for (size_t i = 0; i < n; ++i) {
    const size_t d = internal ? i : o[i];
    ax[d] = a[i].x;
    ay[d] = a[i].y;
    az[d] = a[i].z;
    pot[d] = a[i].w;
  }
  return NB_OK;
}

int nb_neighbour_lists(nb_ctx* c, double h_list) {
  if (!c) return NB_ERR_INPUT;
  if (!(h_list >= 0.0) || !std::isfinite(h_list))
    return set_err(c, NB_ERR_INPUT, "search radius must be finite and >= 0");
  if (!c->tree_valid || !c->positions_fresh)
    return set_err(c, NB_ERR_STATE,
                   "neighbour lists need a tree of the current positions");
  c->nbr_valid = c->rho_valid = false;
  int rc;
  {
    Timed t(c, NB_PH_WALK);
    if ((rc = launch_nbr_count(c, h_list))) return rc;
    if ((rc = launch_xcd_plan(c, true))) return rc;
  }
  // totals, the work-item count of the tree's groups (the density kernel
  // runs on the force kernel's work items) and the density launch plan
  if ((rc = stage_d2h(c, 64, c->xcd_plan.p, 9 * 8))) return rc;
  if ((rc = stage_d2h(c, 0, c->nb_off.p + c->n_groups, 8))) return rc;
  if ((rc = stage_d2h(c, 8, c->nb_toff.p + c->n_groups, 8))) return rc;
  if ((rc = stage_d2h(c, 16, c->g_chunks.p + c->n_groups, 4))) return rc;
  if ((rc = sync(c))) return rc;
  const uint64_t* hs = static_cast<const uint64_t*>(c->h_small);
  c->n_nbr = (int64_t)hs[0];
  const int64_t n_tok = (int64_t)hs[1];
  c->n_wi = static_cast<const uint32_t*>(c->h_small)[4];
  for (int x = 0; x <= 8; ++x) c->nbr_b[x] = (int64_t)hs[8 + x];
  if ((rc = reserve(c, c->nb_ids, (size_t)c->n_nbr + 1))) return rc;
  if ((rc = reserve(c, c->tok, (size_t)n_tok + 1))) return rc;
  {
    Timed t(c, NB_PH_WALK);
    if ((rc = launch_nbr_fill(c, h_list))) return rc;
  }
  c->nbr_h = h_list;
  c->nbr_valid = true;
  return NB_OK;
}

int nb_sph_density(nb_ctx* c, double h) {
  if (!c) return NB_ERR_INPUT;
  if (!c->nbr_valid) return set_err(c, NB_ERR_STATE, "no neighbour lists");
  if (!(h > 0.0) || !(h <= c->nbr_h))
    return set_err(c, NB_ERR_INPUT,
                   "h must be > 0 and at most the lists' search radius");
  c->rho_valid = false;
  int rc;
  {
    Timed t(c, NB_PH_FORCE);
    rc = launch_density(c, h);
  }
  if (rc) return rc;
  c->rho_valid = true;
  return NB_OK;
}

int nb_get_density(nb_ctx* c, double* rho, int internal) {
  if (!c) return NB_ERR_INPUT;
  if (!rho) return set_err(c, NB_ERR_INPUT, "NULL output array");
  if (!c->rho_valid) return set_err(c, NB_ERR_STATE, "no density computed");
  const size_t n = (size_t)c->n;
  std::vector<float> a(n);
  std::vector<uint32_t> o(n);
  int rc = sync(c);
  if (!rc) rc = hip_check(c, hipMemcpy(a.data(), c->rho.p, n * sizeof(float),
                                       hipMemcpyDeviceToHost), "rho readback");
  if (!rc) rc = hip_check(c, hipMemcpy(o.data(), c->orig.p, n * 4,
                                       hipMemcpyDeviceToHost), "orig readback");
  if (rc) return rc;
  for (size_t i = 0; i < n; ++i) rho[internal ? i : o[i]] = a[i];
  return NB_OK;
}

int nb_get_neighbour_lists(nb_ctx* c, int64_t* n_entries, int64_t* off,
                           uint32_t* ids) {
  if (!c) return NB_ERR_INPUT;
  if (!c->nbr_valid) return set_err(c, NB_ERR_STATE, "no neighbour lists");
  if (n_entries) *n_entries = c->n_nbr;
  int rc = sync(c);
  if (!rc && off)
    rc = hip_check(c, hipMemcpy(off, c->nb_off.p,
                                ((size_t)c->n_groups + 1) * 8,
                                hipMemcpyDeviceToHost), "list readback");
  if (!rc && ids && c->n_nbr > 0)
    rc = hip_check(c, hipMemcpy(ids, c->nb_ids.p, (size_t)c->n_nbr * 4,
                                hipMemcpyDeviceToHost), "list readback");
  return rc;
}

int nb_get_state(nb_ctx* c, double* x, double* y, double* z, double* vx,
                 double* vy, double* vz, int internal) {
  if (!c) return NB_ERR_INPUT;
  if (!x || !y || !z || !vx || !vy || !vz)
    return set_err(c, NB_ERR_INPUT, "NULL output array");
  if (!c->have_particles) return set_err(c, NB_ERR_STATE, "no particles set");
  const size_t n = (size_t)c->n;
  std::vector<double4> p(n);
  std::vector<double> v[3];
  std::vector<uint32_t> o(n);
  for (auto& a : v) a.resize(n);
  int rc = sync(c);
  if (!rc) rc = hip_check(c, hipMemcpy(p.data(), c->pos.p, n * sizeof(double4),
                                       hipMemcpyDeviceToHost), "pos readback");
  if (!rc) rc = hip_check(c, hipMemcpy(v[0].data(), c->vx.p, n * 8,
                                       hipMemcpyDeviceToHost), "vx readback");
  if (!rc) rc = hip_check(c, hipMemcpy(v[1].data(), c->vy.p, n * 8,
                                       hipMemcpyDeviceToHost), "vy readback");
  if (!rc) rc = hip_check(c, hipMemcpy(v[2].data(), c->vz.p, n * 8,
                                       hipMemcpyDeviceToHost), "vz readback");
  if (!rc) rc = hip_check(c, hipMemcpy(o.data(), c->orig.p, n * 4,
                                       hipMemcpyDeviceToHost), "orig readback");
  if (rc) return rc;
  for (size_t i = 0; i < n; ++i) {
    const size_t d = internal ? i : o[i];
    x[d] = p[i].x;
    y[d] = p[i].y;
    z[d] = p[i].z;
    vx[d] = v[0][i];
    vy[d] = v[1][i];
    vz[d] = v[2][i];
  }
  return NB_OK;
}

int nb_get_info(nb_ctx* c, int64_t* info) {
  if (!c || !info) return NB_ERR_INPUT;
  // refresh mode: list sizes and the evaluated interactions are counted on
  // the device (a refresh changes the lists without the host)
  uint64_t d[kRedCount] = {0};
  if (c->learn && c->red.p) {
    int rc = stage_d2h(c, 0, c->red.p, sizeof d);
    if (!rc) rc = sync(c);
    if (rc) return rc;
    std::memcpy(d, c->h_small, sizeof d);
  }
  const bool dev = c->learn && c->red.p;
  info[0] = c->n;
  info[1] = c->tree_valid ? c->n_cell : 0;
  info[2] = c->tree_valid ? c->n_groups : 0;
  info[3] = c->lists_valid ? (dev ? (int64_t)d[kRedEpj] : c->n_epj) : 0;
  info[4] = c->lists_valid ? (dev ? (int64_t)d[kRedSpj] : c->n_spj) : 0;
  info[5] = c->lists_valid ? (dev ? (int64_t)d[kRedInter] : c->n_inter) : 0;
  info[6] = c->force_evals;
  info[7] = dev ? (int64_t)d[kRedTotInter] : c->total_inter;
  info[8] = c->k;
  info[9] = c->n_wi;
  info[10] = c->n_sys;
  info[11] = dev ? (int64_t)d[kRedRefreshed] : 0;
  info[12] = dev ? (int64_t)d[kRedTotRefreshed] + c->host_refreshed : 0;
  info[13] = c->lists_valid
                 ? (dev ? (int64_t)d[kRedInterSpj] : c->n_inter_spj) : 0;
  info[14] = dev ? (int64_t)d[kRedTotInterSpj] : c->total_inter_spj;
  info[15] = dev ? (int64_t)d[kRedOverflow] : 0;
  info[16] = dev ? (int64_t)d[kRedTotOverflow] : 0;
  return NB_OK;
}

int nb_get_root(nb_ctx* c, double* lo, int32_t* k) {
  if (!c || !lo || !k) return NB_ERR_INPUT;
  if (!c->tree_valid) return set_err(c, NB_ERR_STATE, "no tree");
  Root r;
  int rc = sync(c);
  if (!rc) rc = hip_check(c, hipMemcpy(&r, c->root.p, sizeof r,
                                       hipMemcpyDeviceToHost), "root readback");
  if (rc) return rc;
  for (int a = 0; a < 3; ++a) lo[a] = r.lo[a];
  *k = r.k;
  return NB_OK;
}

int nb_get_roots(nb_ctx* c, double* lo3, int32_t* k) {
  if (!c || !lo3 || !k) return NB_ERR_INPUT;
  if (!c->tree_valid) return set_err(c, NB_ERR_STATE, "no tree");
  std::vector<Root> r((size_t)c->n_sys);
  int rc = sync(c);
  if (!rc) rc = hip_check(c, hipMemcpy(r.data(), c->root.p,
                                       r.size() * sizeof(Root),
                                       hipMemcpyDeviceToHost), "root readback");
  if (rc) return rc;
  for (size_t s = 0; s < r.size(); ++s) {
    for (int a = 0; a < 3; ++a) lo3[3 * s + a] = r[s].lo[a];
    k[s] = r[s].k;
  }
  return NB_OK;
}

int nb_get_keys(nb_ctx* c, uint64_t* key, uint32_t* orig) {
  if (!c) return NB_ERR_INPUT;
  if (!c->tree_valid) return set_err(c, NB_ERR_STATE, "no tree");
  int rc = sync(c);
  if (!rc && key)
    rc = hip_check(c, hipMemcpy(key, c->key.p, (size_t)c->n * 8,
                                hipMemcpyDeviceToHost), "key readback");
  if (!rc && orig)
    rc = hip_check(c, hipMemcpy(orig, c->orig.p, (size_t)c->n * 4,
                                hipMemcpyDeviceToHost), "orig readback");
  return rc;
}

int nb_get_cells(nb_ctx* c, uint8_t* level, uint32_t* begin, uint32_t* count,
                 uint32_t* parent, uint32_t* skip, uint8_t* leaf,
                 double* ctr3) {
  if (!c) return NB_ERR_INPUT;
  if (!c->tree_valid) return set_err(c, NB_ERR_STATE, "no tree");
  const size_t nc = (size_t)c->n_cell;
  std::vector<CellRec> r(nc);
  int rc = sync(c);
  if (!rc) rc = hip_check(c, hipMemcpy(r.data(), c->c_rec.p,
                                       nc * sizeof(CellRec),
                                       hipMemcpyDeviceToHost), "cell readback");
  if (rc) return rc;
  for (size_t i = 0; i < nc; ++i) {
    const uint4 m = r[i].meta;
    if (level) level[i] = (uint8_t)(m.w & 255u);
    if (begin) begin[i] = m.x;
    if (count) count[i] = m.y - m.x;
    if (parent) parent[i] = r[i].aux.x;
    if (skip) skip[i] = m.z;
    if (leaf) leaf[i] = (uint8_t)((m.w >> 8) & 1u);
    if (ctr3) {
      ctr3[3 * i] = r[i].geo.x;
      ctr3[3 * i + 1] = r[i].geo.y;
      ctr3[3 * i + 2] = r[i].geo.z;
    }
  }
  return NB_OK;
}

int nb_get_moments(nb_ctx* c, double* mass, double* com3, double* quad6) {
  if (!c) return NB_ERR_INPUT;
  if (!c->tree_valid) return set_err(c, NB_ERR_STATE, "no tree");
  const size_t nc = (size_t)c->n_cell;
  std::vector<double4> pm(nc);
  std::vector<float4> q(2 * nc);
  int rc = sync(c);
  if (!rc) rc = hip_check(c, hipMemcpy(pm.data(), c->c_pm.p, nc * 32,
                                       hipMemcpyDeviceToHost), "moment readback");
  if (!rc && quad6 && c->cfg.order == 2)
    rc = hip_check(c, hipMemcpy(q.data(), c->c_quad.p, nc * 32,
                                hipMemcpyDeviceToHost), "moment readback");
  if (rc) return rc;
  for (size_t i = 0; i < nc; ++i) {
    if (mass) mass[i] = pm[i].w;
    if (com3) {
      com3[3 * i] = pm[i].x;
      com3[3 * i + 1] = pm[i].y;
      com3[3 * i + 2] = pm[i].z;
    }
    if (quad6) {
      const bool qd = c->cfg.order == 2;
      const float4 a = qd ? q[2 * i] : make_float4(0.f, 0.f, 0.f, 0.f);
      const float4 b = qd ? q[2 * i + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
      const double v[6] = {a.x, a.y, a.z, a.w, b.x, b.y};
      for (int k = 0; k < 6; ++k) quad6[6 * i + k] = v[k];
    }
  }
  return NB_OK;
}

int nb_get_groups(nb_ctx* c, uint32_t* cell, uint32_t* begin, uint32_t* count,
                  double* lo3, double* hi3, double* ctr3) {
  if (!c) return NB_ERR_INPUT;
  if (!c->tree_valid) return set_err(c, NB_ERR_STATE, "no tree");
  const size_t ng = (size_t)c->n_groups;
  std::vector<uint32_t> gc(ng), gb(ng), gn(ng);
  std::vector<double4> lo(ng), hi(ng);
  int rc = sync(c);
  if (!rc) rc = hip_check(c, hipMemcpy(gc.data(), c->g_cell.p, ng * 4,
                                       hipMemcpyDeviceToHost), "group readback");
  if (!rc) rc = hip_check(c, hipMemcpy(gb.data(), c->g_begin.p, ng * 4,
                                       hipMemcpyDeviceToHost), "group readback");
  if (!rc) rc = hip_check(c, hipMemcpy(gn.data(), c->g_count.p, ng * 4,
                                       hipMemcpyDeviceToHost), "group readback");
  if (!rc) rc = hip_check(c, hipMemcpy(lo.data(), c->g_lo.p, ng * 32,
                                       hipMemcpyDeviceToHost), "group readback");
  if (!rc) rc = hip_check(c, hipMemcpy(hi.data(), c->g_hi.p, ng * 32,
                                       hipMemcpyDeviceToHost), "group readback");
  if (rc) return rc;
  std::vector<CellRec> rec;
  if (ctr3) {
    rec.resize((size_t)c->n_cell);
    rc = hip_check(c, hipMemcpy(rec.data(), c->c_rec.p,
                                rec.size() * sizeof(CellRec),
                                hipMemcpyDeviceToHost), "group readback");
    if (rc) return rc;
  }
  for (size_t g = 0; g < ng; ++g) {
    if (cell) cell[g] = gc[g];
    if (begin) begin[g] = gb[g];
    if (count) count[g] = gn[g];
    if (lo3) {
      lo3[3 * g] = lo[g].x;
      lo3[3 * g + 1] = lo[g].y;
      lo3[3 * g + 2] = lo[g].z;
    }
    if (hi3) {
      hi3[3 * g] = hi[g].x;
      hi3[3 * g + 1] = hi[g].y;
      hi3[3 * g + 2] = hi[g].z;
    }
    if (ctr3) {
      ctr3[3 * g] = rec[gc[g]].geo.x;
      ctr3[3 * g + 1] = rec[gc[g]].geo.y;
      ctr3[3 * g + 2] = rec[gc[g]].geo.z;
    }
  }
  return NB_OK;
}

int nb_upload_lists(nb_ctx* c, int64_t n_groups, const int64_t* epj_off,
                    int64_t n_epj, const uint32_t* epj,
                    const int64_t* spj_off, int64_t n_spj,
                    const uint32_t* spj, int on_device) {
  if (!c) return NB_ERR_INPUT;
  if (!c->tree_valid)
    return set_err(c, NB_ERR_STATE, "uploaded lists need a built tree");
  if (c->learn)
    return set_err(c, NB_ERR_STATE,
                   "uploaded lists carry no walk state for refresh mode");
  if (n_groups != c->n_groups)
    return set_err(c, NB_ERR_INPUT, "group count %lld, the tree has %lld",
                   (long long)n_groups, (long long)c->n_groups);
  if (!epj_off || !spj_off || (n_epj > 0 && !epj) || (n_spj > 0 && !spj))
    return set_err(c, NB_ERR_INPUT, "NULL list array");
  if (n_epj < 0 || n_spj < 0 || n_epj >= (int64_t)1 << 40 ||
      n_spj >= (int64_t)1 << 40)
    return set_err(c, NB_ERR_INPUT, "list totals out of range");
  drop_graph(c);
  c->lists_valid = c->lists_reusable = false;
  c->tail.valid = false;
  const size_t ng = (size_t)c->n_groups;
  int rc = reserve(c, c->epj_off, ng + 1);
  if (!rc) rc = reserve(c, c->spj_off, ng + 1);
  if (!rc) rc = reserve(c, c->epj, (size_t)n_epj + 1);
  if (!rc) rc = reserve(c, c->spj, (size_t)n_spj + 1);
  if (!rc) rc = reserve(c, c->cnt_e, ng);
  if (!rc) rc = reserve(c, c->cnt_s, ng);
  if (!rc) rc = reserve(c, c->lflag, 1);
  if (rc) return rc;
  const hipMemcpyKind kind =
      on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  rc = hip_check(c, hipMemcpyAsync(c->epj_off.p, epj_off, (ng + 1) * 8, kind,
                                   c->stream), "list upload");
  if (!rc)
    rc = hip_check(c, hipMemcpyAsync(c->spj_off.p, spj_off, (ng + 1) * 8,
                                     kind, c->stream), "list upload");
  if (!rc && n_epj)
    rc = hip_check(c, hipMemcpyAsync(c->epj.p, epj, (size_t)n_epj * 4, kind,
                                     c->stream), "list upload");
  if (!rc && n_spj)
    rc = hip_check(c, hipMemcpyAsync(c->spj.p, spj, (size_t)n_spj * 4, kind,
                                     c->stream), "list upload");
  if (!rc) rc = fill_u32(c, c->lflag.p, 1, 0u);
  if (rc) return rc;
  c->n_epj = n_epj;
  c->n_spj = n_spj;
  // validate before anything indexes with the ids
  if ((rc = launch_check_lists(c, c->lflag.p))) return rc;
  if ((rc = stage_d2h(c, 0, c->lflag.p, 4))) return rc;
  if ((rc = sync(c))) return rc;
  const unsigned bad = *static_cast<const unsigned*>(c->h_small);
  if (bad) {
    c->n_epj = c->n_spj = 0;
    return set_err(c, NB_ERR_LIST,
                   "uploaded lists rejected:%s%s%s%s",
                   (bad & 1) ? " bad EPJ offsets" : "",
                   (bad & 2) ? " bad SPJ offsets" : "",
                   (bad & 4) ? " EPJ id >= n" : "",
                   (bad & 8) ? " SPJ id >= cells" : "");
  }
  if ((rc = launch_interactions(c, c->cnt_e.p, c->cnt_s.p))) return rc;
  if ((rc = launch_xcd_plan(c, false))) return rc;
  if ((rc = stage_d2h(c, 64, c->xcd_plan.p, 9 * 8))) return rc;
  if ((rc = stage_d2h(c, 16, c->red.p, 8))) return rc;
  if ((rc = stage_d2h(c, 40, c->g_chunks.p + c->n_groups, 4))) return rc;
  if ((rc = stage_d2h(c, 48, c->red.p + 2, 8))) return rc;
  if ((rc = sync(c))) return rc;
  {
    const uint64_t* h = static_cast<const uint64_t*>(c->h_small);
    c->n_inter = (int64_t)h[2];
    c->n_inter_spj = (int64_t)h[6];
    c->n_wi = static_cast<const uint32_t*>(c->h_small)[10];
    for (int x = 0; x <= 8; ++x) c->xcd_b[x] = (int64_t)h[8 + x];
    if (c->learn) c->lane_total = (int64_t)h[20];
  }
  if ((rc = launch_tail_order(c))) return rc;
  c->lists_valid = true;
  c->lists_reusable = true;
  return NB_OK;
}

int nb_get_lists(nb_ctx* c, int64_t* epj_off, uint32_t* epj,
                 int64_t* spj_off, uint32_t* spj) {
  if (!c) return NB_ERR_INPUT;
  if (!c->lists_valid) return set_err(c, NB_ERR_STATE, "no lists");
  const size_t ng = (size_t)c->n_groups;
  int rc = sync(c);
  if (!rc && c->learn) {
    // refresh mode: each list sits at the start of a slot with room to grow;
    // read slots and lengths and pack the lists into CSR
    std::vector<uint64_t> eo(ng + 1), so(ng + 1);
    std::vector<uint32_t> ne(ng), ns(ng), e((size_t)c->cap_e + 1),
        s((size_t)c->cap_s + 1);
    rc = hip_check(c, hipMemcpy(eo.data(), c->epj_off.p, (ng + 1) * 8,
                                hipMemcpyDeviceToHost), "list readback");
    if (!rc) rc = hip_check(c, hipMemcpy(so.data(), c->spj_off.p, (ng + 1) * 8,
                                         hipMemcpyDeviceToHost), "list readback");
    if (!rc) rc = hip_check(c, hipMemcpy(ne.data(), c->cnt_e.p, ng * 4,
                                         hipMemcpyDeviceToHost), "list readback");
    if (!rc) rc = hip_check(c, hipMemcpy(ns.data(), c->cnt_s.p, ng * 4,
                                         hipMemcpyDeviceToHost), "list readback");
    if (!rc && epj) rc = hip_check(c, hipMemcpy(e.data(), c->epj.p,
                                                (size_t)c->cap_e * 4,
                                                hipMemcpyDeviceToHost),
                                   "list readback");
    if (!rc && spj) rc = hip_check(c, hipMemcpy(s.data(), c->spj.p,
                                                (size_t)c->cap_s * 4,
                                                hipMemcpyDeviceToHost),
                                   "list readback");
    if (rc) return rc;
    int64_t oe = 0, os = 0;
    for (size_t g = 0; g < ng; ++g) {
      if (epj_off) epj_off[g] = oe;
      if (spj_off) spj_off[g] = os;
      if (epj) std::copy(e.begin() + eo[g], e.begin() + eo[g] + ne[g], epj + oe);
      if (spj) std::copy(s.begin() + so[g], s.begin() + so[g] + ns[g], spj + os);
      oe += ne[g];
      os += ns[g];
    }
    if (epj_off) epj_off[ng] = oe;
    if (spj_off) spj_off[ng] = os;
    return NB_OK;
  }
  if (!rc && epj_off)
    rc = hip_check(c, hipMemcpy(epj_off, c->epj_off.p, (ng + 1) * 8,
                                hipMemcpyDeviceToHost), "list readback");
  if (!rc && spj_off)
    rc = hip_check(c, hipMemcpy(spj_off, c->spj_off.p, (ng + 1) * 8,
                                hipMemcpyDeviceToHost), "list readback");
  if (!rc && epj && c->n_epj)
    rc = hip_check(c, hipMemcpy(epj, c->epj.p, (size_t)c->n_epj * 4,
                                hipMemcpyDeviceToHost), "list readback");
  if (!rc && spj && c->n_spj)
    rc = hip_check(c, hipMemcpy(spj, c->spj.p, (size_t)c->n_spj * 4,
                                hipMemcpyDeviceToHost), "list readback");
  return rc;
}

int nb_get_timing(nb_ctx* c, double* ms, int64_t* calls, int reset) {
  if (!c || !ms) return NB_ERR_INPUT;
  resolve_timers(c);
  for (int p = 0; p < NB_PH_COUNT; ++p) {
    ms[p] = c->ph_ms[p];
    if (calls) calls[p] = c->ph_calls[p];
  }
  if (reset) {
    for (int p = 0; p < NB_PH_COUNT; ++p) {
      c->ph_ms[p] = 0.0;
      c->ph_calls[p] = 0;
    }
  }
  return NB_OK;
}

}  // extern "C"
