// C ABI: argument checks, plan lifecycle and dispatch.  Every numerical step
// runs in the device kernels of the other translation units.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "../../include/bemfmm.h"
#include "plan.h"

namespace bemfmm {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

int objective_grad(Problem& P, const c64* beta, const double* dir, const double* pts_host,
                   int n_pts, const bem_gmres_opts* opts, double* J, c64* grad, c64* p_out,
                   bem_gmres_info* info_f, bem_gmres_info* info_a, hipStream_t s);
int objective_forward(Problem& P, const c64* beta, const double* dir, const double* pts_host,
                      int n_pts, const bem_gmres_opts* opts, double* J, c64* p_out,
                      c64* pobs_out, bem_gmres_info* info_f, hipStream_t s);
int objective_backward(Problem& P, const c64* beta, const c64* p, const c64* pobs,
                       const double* pts_host, int n_pts, const bem_gmres_opts* opts, c64* grad,
                       bem_gmres_info* info_a, hipStream_t s);
int gmres_solve_batch(std::vector<Problem*>& probs, const std::vector<int>& adjoint,
                      const std::vector<const c64*>& sigma, const std::vector<const c64*>& b,
                      const std::vector<c64*>& x, double tol, int m, int max_iter, int mode,
                      double inner_tol, int use_x0, bem_gmres_info* infos, hipStream_t caller);

static void destroy_problem(Problem* P) {
  if (!P) return;
  release_workspace(*P);
  for (hipEvent_t e : P->ev_pool) (void)hipEventDestroy(e);
  P->ev_pool.clear();
  if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
  if (P->ev_join) (void)hipEventDestroy(P->ev_join);
  if (P->own_streams && P->side) (void)hipStreamDestroy(P->side);
  if (P->ev_fork2) (void)hipEventDestroy(P->ev_fork2);
  if (P->ev_join2) (void)hipEventDestroy(P->ev_join2);
  if (P->own_streams && P->side2) (void)hipStreamDestroy(P->side2);
  P->f64.ops.release();
  P->f32.ops.release();
  P->f64.leafops.release();
  P->f32.leafops.release();
  P->f64.release_tcache();
  P->f32.release_tcache();
  P->arena.release();
  delete P;
}

}  // namespace bemfmm

using namespace bemfmm;

struct bem_plan {
  std::vector<Problem*> probs;
  // the side streams of every product of the plan (near field, leaf-level
  // M2L) and of its batched solves: created before anything else of the
  // plan, so that the runtime gives them hardware queues of their own rather
  // than one it already uses for the caller's stream (work on streams that
  // share a queue runs one launch after another)
  hipStream_t side = nullptr, side2 = nullptr;
};

static void destroy_plan(bem_plan* plan) {
  for (Problem* P : plan->probs) destroy_problem(P);
  if (plan->side) (void)hipStreamDestroy(plan->side);
  if (plan->side2) (void)hipStreamDestroy(plan->side2);
  delete plan;
}

static int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

static Problem* get_prob(bem_plan* plan, int prob) {
  if (!plan || prob < 0 || prob >= (int)plan->probs.size()) return nullptr;
  return plan->probs[prob];
}

// Mean time of one product of a built problem (HIP events), float32 or float64.
static int time_product(Problem& P, bool f32, hipStream_t s, float* ms) {
  c64* v = nullptr;
  c64* y = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (v) (void)hipFree(v);
    if (y) (void)hipFree(y);
  };
  int r = 0;
  auto check = [&](hipError_t e) {
    if (e != hipSuccess && !r) {
      set_error(std::string("HIP error '") + hipGetErrorString(e) + "' in the leaf-level tuner");
      r = -3;
    }
    return r == 0;
  };
  if (check(hipMalloc((void**)&v, sizeof(c64) * P.n)) &&
      check(hipMalloc((void**)&y, sizeof(c64) * P.n)) &&
      check(hipMemsetAsync(v, 0, sizeof(c64) * P.n, s)) && check(hipEventCreate(&e0)) &&
      check(hipEventCreate(&e1))) {
    auto apply = [&]() {
      return f32 ? fmm_apply<float>(P, P.f32, v, nullptr, y, s)
                 : fmm_apply<double>(P, P.f64, v, nullptr, y, s);
    };
    r = apply();  // warm-up
    if (!r) check(hipEventRecord(e0, s));
    for (int t = 0; t < 5 && !r; ++t) r = apply();
    float t = 0.f;
    if (!r && check(hipEventRecord(e1, s)) && check(hipEventSynchronize(e1)) &&
        check(hipEventElapsedTime(&t, e0, e1)))
      *ms = t / 5.0f;
  }
  cleanup();
  return r;
}

// Autotuner: the leaf level chosen by the occupancy rule and its two
// neighbours (within [2, finest level allowed by the near radius]) are built
// and timed on a float32 product; the fastest plan is kept.
// Stream schedule per precision: each candidate is timed on the problem's
// own products and the fastest kept (the products' results do not depend on
// the schedule).
// Then, per level, dense or rotation-based M2L (rotation tables built here),
// and the pair-tile width of the leaf-level M2L where it stays dense (its
// width from the tile-count rule and the other widths).
// Then, for the kept schedule, the grids of the two large launches that run
// beside the far-field chain: the near field (one workgroup per leaf, or a
// grid-stride launch of 2 or 4 per compute unit) and the leaf-level M2L (one
// per tile, or 1 or 2 per compute unit).
// A candidate replaces the current choice only when more than 2% faster
// (timings of a few products vary by about that much).
template <typename R>
static int tune_rotations(Problem& P, PrecisionData<R>& D, int prec, hipStream_t s, float gain,
                          float* best_ms) {
  int r = build_rotations<R>(P, D, s);
  if (r) return r;
  for (int l = P.L; l >= 2; --l) {
    GroupedOp<R>& op = D.m2l[l];
    if (!op.rot_ready) continue;
    op.rot_on = true;
    if (P.m2l_rot_req == 2) continue;  // requested wherever the order allows
    float ms = 0.f;
    if ((r = time_product(P, prec == 1, s, &ms))) return r;
    if (ms < gain * *best_ms)
      *best_ms = ms;
    else
      op.rot_on = false;
  }
  if (P.m2l_rot_req == 2) return time_product(P, prec == 1, s, best_ms);
  return 0;
}

template <typename R>
static int tune_leaf_tile(Problem& P, PrecisionData<R>& D, int prec, hipStream_t s, float gain,
                          float* best_ms) {
  GroupedOp<R>& op = D.m2l[P.L];
  if (op.rot_on || op.n_pairs == 0) return 0;
  const int first = op.ct;
  int best = first;
  for (int ct : {128, 64, 32, 16}) {
    if (ct == first || (ct == 128 && sizeof(R) == 8)) continue;
    int r = retile_forward<R>(op, ct, D.ops, s);
    float ms = 0.f;
    if (!r) r = time_product(P, prec == 1, s, &ms);
    if (r) return r;
    if (ms < gain * *best_ms) {
      *best_ms = ms;
      best = ct;
    }
  }
  return retile_forward<R>(op, best, D.ops, s);
}

static int tune_schedule(Problem& P, hipStream_t s) {
  int dev = 0, ncu = 0;
  BEM_HIP_TRY(hipGetDevice(&dev));
  BEM_HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const float gain = 0.98f;
  for (int prec = 0; prec < 2; ++prec) {
    const int nd_max = prec == 1 ? P.f32.n_direct : P.f64.n_direct;
    int best = 0;
    float best_ms = 0.f;
    P.p2p_cap[prec] = 0;
    P.m2l_cap[prec] = 0;
    P.ndir[prec] = 0;
    for (int c = 0; c < SCHED_COUNT; ++c) {
      P.sched[prec] = c;
      float ms = 0.f;
      int r = time_product(P, prec == 1, s, &ms);
      if (r) return r;
      if (c == 0 || ms < gain * best_ms) {
        best = c;
        best_ms = ms;
      }
    }
    P.sched[prec] = best;
    // direct leaf <-> ancestor translations instead of the chains
    if (nd_max > 0) {
      P.ndir[prec] = nd_max;
      float ms = 0.f;
      int r = time_product(P, prec == 1, s, &ms);
      if (r) return r;
      if (ms < gain * best_ms)
        best_ms = ms;
      else
        P.ndir[prec] = 0;
    }
    // multipole-to-local by rotation, level by level from the leaves up
    if (P.m2l_rot_req != 1) {
      int r = prec == 1 ? tune_rotations<float>(P, P.f32, prec, s, gain, &best_ms)
                        : tune_rotations<double>(P, P.f64, prec, s, gain, &best_ms);
      if (r) return r;
    }
    // pair-tile width of the leaf-level M2L where it runs the dense kernel
    {
      int r = prec == 1 ? tune_leaf_tile<float>(P, P.f32, prec, s, gain, &best_ms)
                        : tune_leaf_tile<double>(P, P.f64, prec, s, gain, &best_ms);
      if (r) return r;
    }
    // near-field grid x leaf-level M2L grid (one or two workgroups per CU)
    int best_p = 0, best_m = 0;
    P.m2l_cap[prec] = 0;
    for (int pm : {0, 2, 4})
      for (int mm : {0, 1, 2}) {
        if (pm == 0 && mm == 0) continue;  // timed above
        const int pc = pm * ncu, mc = mm * ncu;
        if (pc >= P.nbox[P.L]) continue;
        P.p2p_cap[prec] = pc;
        P.m2l_cap[prec] = mc;
        float ms = 0.f;
        int r = time_product(P, prec == 1, s, &ms);
        if (r) return r;
        if (ms < gain * best_ms) {
          best_p = pc;
          best_m = mc;
          best_ms = ms;
        }
      }
    P.p2p_cap[prec] = best_p;
    P.m2l_cap[prec] = best_m;
  }
  return 0;
}

namespace bemfmm {

// Order calibration of one precision.  The level rule's orders are shifted
// until the sampled relative error of the product, the larger of its
// white-noise and plane-wave errors, is below 0.7 of the tolerance (the
// factor covers the spread of the sampled estimate): all levels by the same
// amount first (error per order step: ~x1.9 on the workloads measured, so a
// step up is estimated with that rate and a step down with 2.2, then
// checked), then the leaf level alone and the coarser levels alone are
// lowered one order at a time while the target still holds (the leaf level
// holds most of the pairs, so its order sets most of the cost).  The float64
// orders may move below the rule; the float32 ones are only raised (the
// mixed-precision refinement's step count rests on the rule's float32
// accuracy).
template <typename R>
static int calibrate_one(Problem& P, PrecisionData<R>& D, double tol, bool may_lower,
                         hipStream_t s) {
  double e = 0;
  int r = measure_error<R>(P, D, s, &e);
  if (r) return r;
  const int req = sizeof(R) == 8 ? P.order64_req : P.order32_req;
  if (!(tol > 0) || req > 0) return 0;
  const double target = 0.7 * tol;
  auto top = [&]() {
    int pm = 0;
    for (int l = 2; l <= P.L; ++l) pm = std::max(pm, D.order[l]);
    return pm;
  };
  auto lowest = [&]() {
    int pm = 1 << 20;
    for (int l = 2; l <= P.L; ++l) pm = std::min(pm, D.order[l]);
    return pm;
  };
  int sc = D.shift_c, sl = D.shift;
  auto build = [&](int c, int l, double* ee) -> int {
    int rr = rebuild_precision<R>(P, D, c, l, s);
    if (!rr) rr = measure_error<R>(P, D, s, ee);
    return rr;
  };
  if (e > target) {
    double prev = e;
    while (e > target && top() < std::min(P.p_max, 40)) {
      const int step = std::max(1, (int)std::ceil(std::log(e / target) / std::log(1.9)));
      sc += step;
      sl += step;
      if ((r = build(sc, sl, &e))) return r;
      if (e > 0.8 * prev && e > target) break;  // rounding floor: higher orders do not help
      prev = e;
    }
    if (e > target) return 0;  // the best the orders allow
  } else if (may_lower && e > 0) {
    const int down = (int)std::floor(std::log(target / e) / std::log(2.2));
    if (down >= 1) {
      double e2 = 0;
      if ((r = build(sc - down, sl - down, &e2))) return r;
      if (e2 <= target) {
        sc -= down;
        sl -= down;
        e = e2;
      }
    }
  }
  // one order less on the leaf level alone, then on the coarser levels
  // alone, while the target holds
  bool built_is_best = D.shift_c == sc && D.shift == sl;
  for (int which = 0; which < 2; ++which) {
    if (which == 1 && P.L <= 2) break;  // no levels above the leaves
    for (;;) {
      const int nc = sc - (which == 1 ? 1 : 0), nl = sl - (which == 0 ? 1 : 0);
      if (!may_lower && (nc < 0 || nl < 0)) break;
      if (lowest() <= 1) break;
      const auto before = D.order;
      double e2 = 0;
      if ((r = build(nc, nl, &e2))) return r;
      built_is_best = e2 <= target;
      if (D.order == before) break;  // no order moved (all at their bound)
      if (!built_is_best) break;
      sc = nc;
      sl = nl;
      e = e2;
    }
  }
  if (!built_is_best && (r = build(sc, sl, &e))) return r;
  // translations across three boxes converge much faster than those across
  // two: drop input orders from them while the target holds
  if (may_lower) {
    int fc = D.far_cut;
    for (;;) {
      double e2 = 0;
      D.far_cut = fc + 1;
      if ((r = build(sc, sl, &e2))) return r;
      if (e2 > target || fc + 1 >= lowest()) {
        D.far_cut = fc;
        if ((r = build(sc, sl, &e))) return r;
        break;
      }
      fc = D.far_cut;
      e = e2;
    }
  }
  return 0;
}

// Without a float32 target the float32 orders stay at the level rule; the
// input cut of the translations across three boxes is still taken as far as
// it leaves both sampled errors within 25% of the uncut ones.
template <typename R>
static int cut_far_relative(Problem& P, PrecisionData<R>& D, hipStream_t s) {
  const double w0 = D.err, s0 = D.err_smooth;
  if (!(w0 > 0) || !(s0 > 0)) return 0;
  int lowest = 1 << 20;
  for (int l = 2; l <= P.L; ++l) lowest = std::min(lowest, D.order[l]);
  int fc = D.far_cut, r = 0;
  for (;;) {
    double e = 0;
    D.far_cut = fc + 1;
    if ((r = rebuild_precision<R>(P, D, D.shift_c, D.shift, s))) return r;
    if ((r = measure_error<R>(P, D, s, &e))) return r;
    if (D.err > 1.25 * w0 || D.err_smooth > 1.25 * s0 || fc + 1 >= lowest) {
      D.far_cut = fc;
      if ((r = rebuild_precision<R>(P, D, D.shift_c, D.shift, s))) return r;
      return measure_error<R>(P, D, s, &e);
    }
    fc = D.far_cut;
  }
}

int calibrate_orders(Problem& P, hipStream_t s) {
  if (P.direct || P.L < 2) return 0;
  int r = calibrate_one<double>(P, P.f64, P.fmm_tol64, true, s);
  if (!r) r = calibrate_one<float>(P, P.f32, P.fmm_tol32, false, s);
  if (!r && !(P.fmm_tol32 > 0) && P.order32_req <= 0) r = cut_far_relative<float>(P, P.f32, s);
  P.f64.release_tcache();
  P.f32.release_tcache();
  return r;
}

}  // namespace bemfmm

template <typename Build>
static int autotune_leaf_level(const bem_problem& q, Build& build_one, Problem** best,
                               hipStream_t s) {
  Problem* cur = *best;
  float best_ms = 0.f;
  int r = time_product(*cur, true, s, &best_ms);
  if (r) return r;
  const int L0 = cur->L;
  for (int L : {L0 - 1, L0 + 1}) {
    if (L < 2) continue;
    Problem* cand = nullptr;
    r = build_one(q, L, &cand);
    if (r) return r;
    if (cand->L != L || cand->direct) {  // level capped by the near radius
      destroy_problem(cand);
      continue;
    }
    float ms = 0.f;
    r = time_product(*cand, true, s, &ms);
    if (r) {
      destroy_problem(cand);
      return r;
    }
    if (ms < best_ms) {
      destroy_problem(*best);
      *best = cand;
      best_ms = ms;
    } else {
      destroy_problem(cand);
    }
  }
  (*best)->tuned_ms = best_ms;
  return 0;
}

extern "C" {

const char* bem_last_error(void) { return g_last_error.c_str(); }

int bem_plan_create(const bem_problem* probs, int n_probs, void* stream, bem_plan** out) {
  if (!out) return fail(BEM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!probs || n_probs < 1) return fail(BEM_E_INVALID, "no problems given");
  for (int i = 0; i < n_probs; ++i) {
    const bem_problem& q = probs[i];
    if (!q.vert || !q.tri) return fail(BEM_E_INVALID, "NULL mesh array");
    if (q.n_tri < 1 || q.n_vert < 3) return fail(BEM_E_INVALID, "empty mesh");
    if (q.n_tri > (int64_t)1 << 28) return fail(BEM_E_INVALID, "mesh too large");
    if (!(q.k > 0.0) || !std::isfinite(q.k)) return fail(BEM_E_INVALID, "wavenumber must be > 0");
    if (!std::isfinite(q.alpha_re) || !std::isfinite(q.alpha_im))
      return fail(BEM_E_INVALID, "non-finite alpha");
    for (int64_t t = 0; t < 3 * q.n_tri; ++t)
      if (q.tri[t] < 0 || q.tri[t] >= q.n_vert)
        return fail(BEM_E_INVALID, "triangle vertex index out of range");
    for (int64_t t = 0; t < 3 * q.n_vert; ++t)
      if (!std::isfinite(q.vert[t])) return fail(BEM_E_INVALID, "non-finite vertex coordinate");
    if (q.order64 > 40 || q.order32 > 40) return fail(BEM_E_INVALID, "expansion order > 40");
    if (!std::isfinite(q.fmm_tol) || !std::isfinite(q.fmm_tol32) || q.fmm_tol >= 1.0 ||
        q.fmm_tol32 >= 1.0)
      return fail(BEM_E_INVALID, "fmm_tol must be finite and < 1");
    if (q.p_max > 40) return fail(BEM_E_INVALID, "p_max > 40");
    if (q.m2l_rot < 0 || q.m2l_rot > 2) return fail(BEM_E_INVALID, "m2l_rot must be 0, 1 or 2");
  }
  hipStream_t s = (hipStream_t)stream;
  bem_plan* plan = new bem_plan();
  if (hipStreamCreateWithFlags(&plan->side, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&plan->side2, hipStreamNonBlocking) != hipSuccess) {
    destroy_plan(plan);
    return fail(BEM_E_HIP, "stream creation failed");
  }
  // device address of the allocation-free product's static buffer (once per
  // device, this device current)
  if (int r = scratch_init_current_device()) {
    destroy_plan(plan);
    return r;
  }
  auto build_one = [&](const bem_problem& q, int leaf_level, Problem** outp) -> int {
    Problem* P = new Problem();
    P->side = plan->side;
    P->side2 = plan->side2;
    P->n = q.n_tri;
    P->k = q.k;
    P->alpha = mk(q.alpha_re, q.alpha_im);
    P->eta = q.near_eta > 0 ? q.near_eta : 2.0;
    P->leaf_cap = q.leaf_cap > 0 ? q.leaf_cap : 64;
    P->leaf_level_req = leaf_level;
    P->order64_req = q.order64;
    P->order32_req = q.order32;
    P->fmm_tol64 = q.fmm_tol;
    P->fmm_tol32 = q.fmm_tol32;
    P->p_max = q.p_max > 0 ? q.p_max : 40;
    P->m2l_rot_req = q.m2l_rot;
    int r = build_geometry_and_tree(*P, q.vert, q.n_vert, q.tri, s);
    if (!r) r = build_near_field(*P, s);
    if (!r) r = build_operators(*P, s);
    if (!r) r = calibrate_orders(*P, s);
    if (r) {
      destroy_problem(P);
      return r;
    }
    *outp = P;
    return 0;
  };
  for (int i = 0; i < n_probs; ++i) {
    const bem_problem& q = probs[i];
    Problem* P = nullptr;
    int r = build_one(q, q.leaf_level > 0 ? q.leaf_level : 0, &P);
    if (!r && q.leaf_level < 0 && !P->direct) r = autotune_leaf_level(q, build_one, &P, s);
    if (!r && !P->direct) r = tune_schedule(*P, s);
    if (r) {
      destroy_plan(plan);
      return r;
    }
    plan->probs.push_back(P);
  }
  *out = plan;
  return BEM_OK;
}

int bem_plan_destroy(bem_plan* plan) {
  if (!plan) return BEM_OK;
  destroy_plan(plan);
  return BEM_OK;
}

int bem_plan_get_stats(const bem_plan* plan, int prob, bem_plan_stats* st) {
  Problem* P = get_prob((bem_plan*)plan, prob);
  if (!P || !st) return fail(BEM_E_INVALID, "bad plan, problem index or stats pointer");
  std::memset(st, 0, sizeof(*st));
  st->n_tri = P->n;
  st->leaf_level = P->L;
  st->n_leaves = P->nbox[P->L];
  st->n_near = P->n_near;
  st->n_p2p_pairs = P->n_p2p_pairs;
  for (int l = 0; l <= MAX_LEVEL; ++l) {
    st->n_m2l[l] = P->n_m2l[l];
    st->n_m2l_far[l] = P->n_m2l_far[l];
    st->order64[l] = P->f64.order[l];
    st->order32[l] = P->f32.order[l];
    st->box_size[l] = P->h[l];
  }
  st->device_bytes = P->arena.bytes + P->f64.ops.bytes + P->f32.ops.bytes +
                     P->f64.leafops.bytes + P->f32.leafops.bytes;
  st->fmm_err64 = P->direct ? 0.0 : P->f64.err;
  st->fmm_err32 = P->direct ? 0.0 : P->f32.err;
  st->fmm_err64_smooth = P->direct ? 0.0 : P->f64.err_smooth;
  st->fmm_err32_smooth = P->direct ? 0.0 : P->f32.err_smooth;
  st->far_cut[0] = P->f64.far_cut;
  st->far_cut[1] = P->f32.far_cut;
  for (int l = 2; l <= P->L && !P->direct; ++l) {
    st->m2l_rot64[l] = P->f64.m2l[l].rot_on ? 1 : 0;
    st->m2l_rot32[l] = P->f32.m2l[l].rot_on ? 1 : 0;
  }
  st->tuned_ms = P->tuned_ms;
  for (int l = 0; l < 22; ++l) st->m2l_tile32[l] = (l <= P->L) ? P->f32.m2l[l].ct : 0;
  st->schedule[0] = P->sched[0];
  st->schedule[1] = P->sched[1];
  st->p2p_grid[0] = P->p2p_cap[0];
  st->p2p_grid[1] = P->p2p_cap[1];
  st->m2l_grid[0] = P->m2l_cap[0];
  st->m2l_grid[1] = P->m2l_cap[1];
  st->direct_depth[0] = P->ndir[0];
  st->direct_depth[1] = P->ndir[1];
  return BEM_OK;
}

int bem_fmm_matvec(bem_plan* plan, int prob, int prec, const void* p, const void* q, void* y,
                   int nrhs, void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P) return fail(BEM_E_INVALID, "bad plan or problem index");
  if (!y) return fail(BEM_E_INVALID, "y is NULL");
  if (y == p || y == q) return fail(BEM_E_INVALID, "y aliases an input");
  if (nrhs < 1) return fail(BEM_E_INVALID, "nrhs < 1");
  if (prec != BEM_C128 && prec != BEM_C64) return fail(BEM_E_INVALID, "bad precision");
  hipStream_t s = (hipStream_t)stream;
  for (int c = 0; c < nrhs; ++c) {
    const c64* pc = p ? (const c64*)p + (int64_t)c * P->n : nullptr;
    const c64* qc = q ? (const c64*)q + (int64_t)c * P->n : nullptr;
    c64* yc = (c64*)y + (int64_t)c * P->n;
    int r = (prec == BEM_C128) ? fmm_apply<double>(*P, P->f64, pc, qc, yc, s)
                               : fmm_apply<float>(*P, P->f32, pc, qc, yc, s);
    if (r) return r;
  }
  return BEM_OK;
}

int bem_fmm_matvec_noalloc(bem_plan* plan, int prob, int prec, const void* p, const void* q,
                           void* y, int nrhs, void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P) return fail(BEM_E_INVALID, "bad plan or problem index");
  if (!y) return fail(BEM_E_INVALID, "y is NULL");
  if (y == p || y == q) return fail(BEM_E_INVALID, "y aliases an input");
  if (nrhs < 1) return fail(BEM_E_INVALID, "nrhs < 1");
  if (prec != BEM_C128 && prec != BEM_C64) return fail(BEM_E_INVALID, "bad precision");
  return fmm_matvec_noalloc(*P, prec == BEM_C128 ? 0 : 1, (const c64*)p, (const c64*)q, (c64*)y,
                            nrhs, (hipStream_t)stream);
}

int bem_fmm_matvec_adjoint(bem_plan* plan, int prob, int prec, const void* y, void* u, void* w,
                           int nrhs, void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P) return fail(BEM_E_INVALID, "bad plan or problem index");
  if (!y) return fail(BEM_E_INVALID, "y is NULL");
  if (!u && !w) return fail(BEM_E_INVALID, "both outputs NULL");
  if (u == y || w == y) return fail(BEM_E_INVALID, "output aliases the input");
  if (nrhs < 1) return fail(BEM_E_INVALID, "nrhs < 1");
  if (prec != BEM_C128 && prec != BEM_C64) return fail(BEM_E_INVALID, "bad precision");
  hipStream_t s = (hipStream_t)stream;
  for (int c = 0; c < nrhs; ++c) {
    const c64* yc = (const c64*)y + (int64_t)c * P->n;
    c64* uc = u ? (c64*)u + (int64_t)c * P->n : nullptr;
    c64* wc = w ? (c64*)w + (int64_t)c * P->n : nullptr;
    int r = (prec == BEM_C128) ? fmm_apply_adjoint<double>(*P, P->f64, yc, uc, wc, s)
                               : fmm_apply_adjoint<float>(*P, P->f32, yc, uc, wc, s);
    if (r) return r;
  }
  return BEM_OK;
}

int bem_gmres_solve(bem_plan* plan, int prob, const void* sigma, int adjoint, const void* b,
                    void* x, const bem_gmres_opts* opts, bem_gmres_info* info, void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P) return fail(BEM_E_INVALID, "bad plan or problem index");
  if (!b || !x || !opts) return fail(BEM_E_INVALID, "NULL b, x or opts");
  if (b == x) return fail(BEM_E_INVALID, "x aliases b");
  if (!(opts->tol > 0.0)) return fail(BEM_E_INVALID, "tol must be > 0");
  if (opts->mode != 0 && opts->mode != 1) return fail(BEM_E_INVALID, "bad mode");
  int m = opts->restart > 0 ? opts->restart : 50;
  if (m > 500) return fail(BEM_E_INVALID, "restart > 500");
  int mi = opts->max_iter > 0 ? opts->max_iter : 2000;
  if (info) std::memset(info, 0, sizeof(*info));
  return gmres_solve(*P, (const c64*)sigma, adjoint, (const c64*)b, (c64*)x, opts->tol, m, mi,
                     opts->mode, opts->inner_tol, opts->use_x0, info, (hipStream_t)stream);
}

int bem_gmres_solve_batch(bem_plan* plan, int n_sys, const int32_t* probs,
                          const void* const* sigma, const int32_t* adjoint, const void* const* b,
                          void* const* x, const bem_gmres_opts* opts, bem_gmres_info* infos,
                          void* stream) {
  if (!plan || n_sys < 1 || !probs || !b || !x || !opts)
    return fail(BEM_E_INVALID, "bad batch arguments");
  if (!(opts->tol > 0.0)) return fail(BEM_E_INVALID, "tol must be > 0");
  if (opts->mode != 0 && opts->mode != 1) return fail(BEM_E_INVALID, "bad mode");
  int m = opts->restart > 0 ? opts->restart : 50;
  if (m > 500) return fail(BEM_E_INVALID, "restart > 500");
  int mi = opts->max_iter > 0 ? opts->max_iter : 2000;
  std::vector<Problem*> ps(n_sys);
  std::vector<int> adj(n_sys);
  std::vector<const c64*> sg(n_sys), bb(n_sys);
  std::vector<c64*> xx(n_sys);
  for (int i = 0; i < n_sys; ++i) {
    ps[i] = get_prob(plan, probs[i]);
    if (!ps[i]) return fail(BEM_E_INVALID, "bad problem index in batch");
    if (!b[i] || !x[i] || b[i] == x[i]) return fail(BEM_E_INVALID, "bad b/x in batch");
    for (int j = 0; j < i; ++j)
      if (x[j] == x[i]) return fail(BEM_E_INVALID, "two systems share one solution vector");
    adj[i] = adjoint ? adjoint[i] : 0;
    sg[i] = sigma ? (const c64*)sigma[i] : nullptr;
    bb[i] = (const c64*)b[i];
    xx[i] = (c64*)x[i];
  }
  return gmres_solve_batch(ps, adj, sg, bb, xx, opts->tol, m, mi, opts->mode, opts->inner_tol,
                           opts->use_x0, infos, (hipStream_t)stream);
}

int bem_plane_wave_rhs(bem_plan* plan, int prob, const double* dir3, void* b, void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P || !dir3 || !b) return fail(BEM_E_INVALID, "bad arguments");
  return plane_wave_rhs(*P, dir3, (c64*)b, (hipStream_t)stream);
}

int bem_point_source_rhs(bem_plan* plan, int prob, const double* src, const void* amp, int n_src,
                         void* b, void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P || !src || !amp || !b || n_src < 1) return fail(BEM_E_INVALID, "bad arguments");
  return point_source_rhs(*P, src, (const c64*)amp, n_src, (c64*)b, (hipStream_t)stream);
}

int bem_eval_field(bem_plan* plan, int prob, const void* p, const void* q, const double* pts,
                   int n_pts, const double* dir3, void* out, void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P || !p || !pts || !out || n_pts < 0) return fail(BEM_E_INVALID, "bad arguments");
  return eval_field(*P, (const c64*)p, (const c64*)q, pts, n_pts, dir3, (c64*)out,
                    (hipStream_t)stream);
}

int bem_eval_field_grad(bem_plan* plan, int prob, const void* p, const void* q,
                        const double* pts, int n_pts, const double* dir3, const double* src,
                        const void* amp, int n_src, void* out, void* grad, void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P || !p || !pts || !out || n_pts < 0) return fail(BEM_E_INVALID, "bad arguments");
  if (src && (!amp || n_src < 1)) return fail(BEM_E_INVALID, "point sources without amplitudes");
  return eval_field_grad(*P, (const c64*)p, (const c64*)q, pts, n_pts, dir3, src,
                         (const c64*)amp, n_src, (c64*)out, (c64*)grad, (hipStream_t)stream);
}

struct bem_field_points {
  FieldPoints* F;
};

struct bem_coupling {
  Problem* P = nullptr;
  DevArena arena;
  double* C = nullptr;   // n x n, row-major
  double* Ct = nullptr;  // its transpose (the adjoint's rows)
  c64* q = nullptr;      // work vector of the coupled product
};

int bem_coupling_create(bem_plan* plan, int prob, const double* nodes, int64_t n_nodes,
                        const int32_t* tets, int64_t n_tets, const int32_t* tri, double lambda,
                        double mu, double rho_s, double rho_f, double omega, void* stream,
                        bem_coupling** out) {
  Problem* P = get_prob(plan, prob);
  if (!P || !out) return fail(BEM_E_INVALID, "bad plan, problem index or output pointer");
  *out = nullptr;
  if (!nodes || !tets || !tri || n_nodes < 4 || n_tets < 1)
    return fail(BEM_E_INVALID, "empty or missing solid mesh");
  if (P->n > 65535)  // dense C and C^T (16 n_tri^2 bytes); one launch row per triangle
    return fail(BEM_E_INVALID, "problem too large for a dense coupling matrix (n_tri > 65535)");
  if (3 * n_nodes > BEM_FEM_MAX_DOF)
    return fail(BEM_E_INVALID, "solid mesh too large for the dense factorisation (3 n_nodes > " +
                                   std::to_string(BEM_FEM_MAX_DOF) + ")");
  if (!(mu > 0) || !(3 * lambda + 2 * mu > 0) || !(rho_s > 0) || !(rho_f > 0) || !(omega > 0) ||
      !std::isfinite(lambda) || !std::isfinite(mu) || !std::isfinite(rho_s) ||
      !std::isfinite(rho_f) || !std::isfinite(omega))
    return fail(BEM_E_INVALID, "bad material or frequency");
  for (int64_t i = 0; i < 3 * n_nodes; ++i)
    if (!std::isfinite(nodes[i])) return fail(BEM_E_INVALID, "non-finite node coordinate");
  for (int64_t i = 0; i < 4 * n_tets; ++i)
    if (tets[i] < 0 || tets[i] >= n_nodes) return fail(BEM_E_INVALID, "tetrahedron node out of range");
  for (int64_t i = 0; i < 3 * P->n; ++i)
    if (tri[i] < 0 || tri[i] >= n_nodes) return fail(BEM_E_INVALID, "triangle node out of range");
  // degenerate elements would reach the device as a zero Jacobian
  auto sub = [&](int32_t a, int32_t b, double* d) {
    for (int c = 0; c < 3; ++c) d[c] = nodes[3 * (int64_t)b + c] - nodes[3 * (int64_t)a + c];
  };
  for (int64_t e = 0; e < n_tets; ++e) {
    const int32_t* t = tets + 4 * e;
    double u[3], v[3], w[3];
    sub(t[0], t[1], u);
    sub(t[0], t[2], v);
    sub(t[0], t[3], w);
    const double det = u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) +
                       u[2] * (v[0] * w[1] - v[1] * w[0]);
    if (!(std::fabs(det) > 0.0)) return fail(BEM_E_INVALID, "tetrahedron of zero volume");
  }
  for (int64_t j = 0; j < P->n; ++j) {
    const int32_t* t = tri + 3 * j;
    double u[3], v[3];
    sub(t[0], t[1], u);
    sub(t[0], t[2], v);
    const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2],
                 cz = u[0] * v[1] - u[1] * v[0];
    if (!(cx * cx + cy * cy + cz * cz > 0.0))
      return fail(BEM_E_INVALID, "boundary triangle of zero area");
  }
  hipStream_t s = (hipStream_t)stream;
  bem_coupling* c = new bem_coupling();
  c->P = P;
  int r = coupling_build(*P, nodes, n_nodes, tets, n_tets, tri, lambda, mu, rho_s, rho_f, omega,
                         c->arena, &c->C, &c->Ct, s);
  if (!r) r = c->arena.alloc((void**)&c->q, sizeof(c64) * P->n);
  if (r) {
    c->arena.release();
    delete c;
    return r;
  }
  *out = c;
  return BEM_OK;
}

int bem_coupling_destroy(bem_coupling* c) {
  if (!c) return BEM_OK;
  c->arena.release();
  delete c;
  return BEM_OK;
}

int bem_coupling_get_matrix(const bem_coupling* c, void* C_out, void* stream) {
  if (!c || !C_out) return fail(BEM_E_INVALID, "bad coupling or output pointer");
  BEM_HIP_TRY(hipMemcpyAsync(C_out, c->C, sizeof(double) * c->P->n * c->P->n,
                             hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return BEM_OK;
}

int bem_coupling_apply(const bem_coupling* c, int transpose, const void* v, void* out,
                       void* stream) {
  if (!c || !v || !out) return fail(BEM_E_INVALID, "bad coupling, v or out");
  if (v == out) return fail(BEM_E_INVALID, "out aliases v");
  return coupling_apply(transpose ? c->Ct : c->C, c->P->n, (const c64*)v, (c64*)out, false,
                        (hipStream_t)stream);
}

int bem_coupled_matvec(bem_coupling* c, int prec, const void* p, void* y, void* stream) {
  if (!c || !p || !y) return fail(BEM_E_INVALID, "bad coupling, p or y");
  if (y == p) return fail(BEM_E_INVALID, "y aliases p");
  if (prec != BEM_C128 && prec != BEM_C64) return fail(BEM_E_INVALID, "bad precision");
  Problem& P = *c->P;
  hipStream_t s = (hipStream_t)stream;
  int r = coupling_apply(c->C, P.n, (const c64*)p, c->q, false, s);
  if (r) return r;
  return (prec == BEM_C128) ? fmm_apply<double>(P, P.f64, (const c64*)p, c->q, (c64*)y, s)
                            : fmm_apply<float>(P, P.f32, (const c64*)p, c->q, (c64*)y, s);
}

int bem_coupled_solve(bem_coupling* c, int adjoint, const void* b, void* x,
                      const bem_gmres_opts* opts, bem_gmres_info* info, void* stream) {
  if (!c || !b || !x || !opts) return fail(BEM_E_INVALID, "NULL coupling, b, x or opts");
  if (b == x) return fail(BEM_E_INVALID, "x aliases b");
  if (!(opts->tol > 0.0)) return fail(BEM_E_INVALID, "tol must be > 0");
  if (opts->mode != 0 && opts->mode != 1) return fail(BEM_E_INVALID, "bad mode");
  const int m = opts->restart > 0 ? opts->restart : 50;
  if (m > 500) return fail(BEM_E_INVALID, "restart > 500");
  const int mi = opts->max_iter > 0 ? opts->max_iter : 2000;
  if (info) std::memset(info, 0, sizeof(*info));
  return gmres_solve(*c->P, nullptr, adjoint, (const c64*)b, (c64*)x, opts->tol, m, mi,
                     opts->mode, opts->inner_tol, opts->use_x0, info, (hipStream_t)stream,
                     c->C, c->Ct);
}

int bem_field_points_create(bem_plan* plan, int prob, int prec, const double* pts,
                            int64_t n_pts, void* stream, bem_field_points** out) {
  Problem* P = get_prob(plan, prob);
  if (!P || !out || n_pts < 0 || (n_pts > 0 && !pts)) return fail(BEM_E_INVALID, "bad arguments");
  *out = nullptr;
  FieldPoints* F = nullptr;
  int r = field_points_create(*P, prec, pts, n_pts, &F, (hipStream_t)stream);
  if (r) return r;
  *out = new bem_field_points{F};
  return BEM_OK;
}

int bem_field_points_destroy(bem_field_points* fp) {
  if (!fp) return BEM_OK;
  field_points_destroy(fp->F);
  delete fp;
  return BEM_OK;
}

int bem_field_points_get_stats(const bem_field_points* fp, bem_field_points_stats* st) {
  if (!fp || !st) return fail(BEM_E_INVALID, "bad arguments");
  const FieldPoints& F = *fp->F;
  const Problem& P = *F.P;
  std::memset(st, 0, sizeof(*st));
  st->n_pts = F.n;
  st->levels = F.L;
  for (int l = 0; l <= MAX_LEVEL; ++l) {
    st->n_box[l] = F.nbox[l];
    st->n_m2l[l] = F.n_m2l[l];
    st->n_m2l_far[l] = F.n_m2l_far[l];
    st->order[l] = F.prec == 0 ? P.f64.order[l] : P.f32.order[l];
  }
  st->n_leaf = F.n_leaf;
  st->n_near_pairs = F.n_near_pairs;
  st->device_bytes = F.arena.bytes;
  st->far_cut = 0;  // point-box translations use full orders
  for (int l = 0; l <= F.L && l <= MAX_LEVEL; ++l)
    st->m2l_rot[l] = (F.prec == 0 ? F.f64.m2l[l].rot_on : F.f32.m2l[l].rot_on) ? 1 : 0;
  return BEM_OK;
}

int bem_eval_field_grad_fmm(bem_field_points* fp, const void* p, const void* q,
                            const double* dir3, const double* src, const void* amp, int n_src,
                            void* out, void* grad, void* stream) {
  if (!fp || !p || (!out && fp->F->n > 0)) return fail(BEM_E_INVALID, "bad arguments");
  if (src && (!amp || n_src < 1)) return fail(BEM_E_INVALID, "point sources without amplitudes");
  return eval_field_grad_fmm(*fp->F, (const c64*)p, (const c64*)q, dir3, src, (const c64*)amp,
                             n_src, (c64*)out, (c64*)grad, (hipStream_t)stream);
}

int bem_topological_derivative(int n_pts, const void* p, const void* grad_p, const void* pt,
                               const void* grad_pt, const bem_material* mat, double* T,
                               void* stream) {
  if (!p || !grad_p || !pt || !grad_pt || !mat || !T || n_pts < 0)
    return fail(BEM_E_INVALID, "bad arguments");
  const bem_material& m = *mat;
  if (!(m.rho_f > 0) || !(m.lam_f > 0) || !(m.rho_s > 0) || !(m.lam_s > 0) || !(m.omega > 0) ||
      !std::isfinite(m.rho_f) || !std::isfinite(m.lam_f) || !std::isfinite(m.omega))
    return fail(BEM_E_INVALID, "material constants must be > 0 (solid ones may be +inf)");
  // 3 (rho_s - rho_f) / (2 rho_s + rho_f) and (Lambda_s - Lambda_f) rho_f omega^2 /
  // (Lambda_s Lambda_f); infinite solid constants give the sound-hard limits
  const double cg = std::isinf(m.rho_s) ? 1.5 : 3.0 * (m.rho_s - m.rho_f) / (2.0 * m.rho_s + m.rho_f);
  const double cv = (std::isinf(m.lam_s) ? 1.0 / m.lam_f : (m.lam_s - m.lam_f) / (m.lam_s * m.lam_f)) *
                    m.rho_f * m.omega * m.omega;
  return topological_derivative(n_pts, (const c64*)p, (const c64*)grad_p, (const c64*)pt,
                                (const c64*)grad_pt, cg, cv, T, (hipStream_t)stream);
}

int bem_eval_field_adjoint(bem_plan* plan, int prob, const double* pts, int n_pts, const void* c,
                           void* rp, void* rq, void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P || !pts || !c || !rp || n_pts < 0) return fail(BEM_E_INVALID, "bad arguments");
  return eval_field_adjoint(*P, pts, n_pts, (const c64*)c, (c64*)rp, (c64*)rq,
                            (hipStream_t)stream);
}

int bem_objective_grad(bem_plan* plan, int prob, const void* beta, const double* dir3,
                       const double* pts, int n_pts, const bem_gmres_opts* opts, double* J,
                       void* grad, void* p_out, bem_gmres_info* info_fwd,
                       bem_gmres_info* info_adj, void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P || !beta || !dir3 || !pts || n_pts < 1 || !opts || !J)
    return fail(BEM_E_INVALID, "bad arguments");
  if (!(opts->tol > 0.0)) return fail(BEM_E_INVALID, "tol must be > 0");
  if (info_fwd) std::memset(info_fwd, 0, sizeof(*info_fwd));
  if (info_adj) std::memset(info_adj, 0, sizeof(*info_adj));
  return objective_grad(*P, (const c64*)beta, dir3, pts, n_pts, opts, J, (c64*)grad, (c64*)p_out,
                        info_fwd, info_adj, (hipStream_t)stream);
}

int bem_objective_forward(bem_plan* plan, int prob, const void* beta, const double* dir3,
                          const double* pts, int n_pts, const bem_gmres_opts* opts, double* J,
                          void* p_out, void* pobs_out, bem_gmres_info* info, void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P || !beta || !dir3 || !pts || n_pts < 1 || !opts || !J)
    return fail(BEM_E_INVALID, "bad arguments");
  if (!(opts->tol > 0.0)) return fail(BEM_E_INVALID, "tol must be > 0");
  if (info) std::memset(info, 0, sizeof(*info));
  return objective_forward(*P, (const c64*)beta, dir3, pts, n_pts, opts, J, (c64*)p_out,
                           (c64*)pobs_out, info, (hipStream_t)stream);
}

int bem_objective_backward(bem_plan* plan, int prob, const void* beta, const void* p,
                           const void* pobs, const double* pts, int n_pts,
                           const bem_gmres_opts* opts, void* grad, bem_gmres_info* info,
                           void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P || !beta || !p || !pobs || !pts || n_pts < 1 || !opts || !grad)
    return fail(BEM_E_INVALID, "bad arguments");
  if (!(opts->tol > 0.0)) return fail(BEM_E_INVALID, "tol must be > 0");
  if (grad == beta || grad == p) return fail(BEM_E_INVALID, "grad aliases an input");
  if (info) std::memset(info, 0, sizeof(*info));
  return objective_backward(*P, (const c64*)beta, (const c64*)p, (const c64*)pobs, pts, n_pts,
                            opts, (c64*)grad, info, (hipStream_t)stream);
}

int bem_tree_export(bem_plan* plan, int prob, void* keys, void* perm, void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P) return fail(BEM_E_INVALID, "bad plan or problem index");
  hipStream_t s = (hipStream_t)stream;
  if (keys)
    BEM_HIP_TRY(hipMemcpyAsync(keys, P->keys_orig, sizeof(uint64_t) * P->n,
                               hipMemcpyDeviceToDevice, s));
  if (perm)
    BEM_HIP_TRY(hipMemcpyAsync(perm, P->perm, sizeof(int) * P->n, hipMemcpyDeviceToDevice, s));
  return BEM_OK;
}

int bem_leaves_export(bem_plan* plan, int prob, void* box_keys, void* start, void* end,
                      void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P) return fail(BEM_E_INVALID, "bad plan or problem index");
  hipStream_t s = (hipStream_t)stream;
  int nl = P->nbox[P->L];
  if (box_keys)
    BEM_HIP_TRY(hipMemcpyAsync(box_keys, P->box_keys[P->L], sizeof(uint64_t) * nl,
                               hipMemcpyDeviceToDevice, s));
  if (start)
    BEM_HIP_TRY(hipMemcpyAsync(start, P->box_start[P->L], sizeof(int) * nl,
                               hipMemcpyDeviceToDevice, s));
  if (end)
    BEM_HIP_TRY(hipMemcpyAsync(end, P->box_start[P->L] + 1, sizeof(int) * nl,
                               hipMemcpyDeviceToDevice, s));
  return BEM_OK;
}

int bem_lists_export(bem_plan* plan, int prob, int level, void* box_keys, void* v_dst,
                     void* v_src, void* u_ptr, void* u_idx, int64_t* n_boxes,
                     int64_t* n_pairs, int64_t* n_u, void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P) return fail(BEM_E_INVALID, "bad plan or problem index");
  if (level < 2 || level > P->L) return fail(BEM_E_INVALID, "level outside 2 .. leaf level");
  hipStream_t s = (hipStream_t)stream;
  const int nb = P->nbox[level];
  const GroupedOp<double>& op = P->f64.m2l[level];
  const int np = P->direct ? 0 : op.n_pairs;
  const bool leaf = level == P->L;
  if (n_boxes) *n_boxes = nb;
  if (n_pairs) *n_pairs = np;
  if (n_u) *n_u = leaf ? P->n_u : 0;
  if (box_keys)
    BEM_HIP_TRY(hipMemcpyAsync(box_keys, P->box_keys[level], sizeof(uint64_t) * nb,
                               hipMemcpyDeviceToDevice, s));
  if (np > 0 && v_dst)
    BEM_HIP_TRY(hipMemcpyAsync(v_dst, op.pair_dst, sizeof(int) * np, hipMemcpyDeviceToDevice, s));
  if (np > 0 && v_src)
    BEM_HIP_TRY(hipMemcpyAsync(v_src, op.pair_src, sizeof(int) * np, hipMemcpyDeviceToDevice, s));
  if (leaf && u_ptr)
    BEM_HIP_TRY(hipMemcpyAsync(u_ptr, P->u_ptr, sizeof(int) * (nb + 1), hipMemcpyDeviceToDevice,
                               s));
  if (leaf && u_idx && P->n_u > 0)
    BEM_HIP_TRY(hipMemcpyAsync(u_idx, P->u_idx, sizeof(int) * P->n_u, hipMemcpyDeviceToDevice,
                               s));
  BEM_HIP_TRY(hipStreamSynchronize(s));
  return BEM_OK;
}

int bem_near_export(bem_plan* plan, int prob, void* ptr, void* col, int64_t* n_near,
                    void* stream) {
  Problem* P = get_prob(plan, prob);
  if (!P) return fail(BEM_E_INVALID, "bad plan or problem index");
  hipStream_t s = (hipStream_t)stream;
  if (n_near) *n_near = P->n_near;
  if (ptr)
    BEM_HIP_TRY(hipMemcpyAsync(ptr, P->near_ptr, sizeof(int) * (P->n + 1),
                               hipMemcpyDeviceToDevice, s));
  if (col && P->n_near > 0)
    BEM_HIP_TRY(hipMemcpyAsync(col, P->near_col, sizeof(int) * P->n_near,
                               hipMemcpyDeviceToDevice, s));
  BEM_HIP_TRY(hipStreamSynchronize(s));
  return BEM_OK;
}

int bem_plan_set_tuning(bem_plan* plan, int prob, int prec, int schedule, int p2p_grid,
                        int m2l_grid, int direct_depth) {
  Problem* P = get_prob(plan, prob);
  if (!P) return fail(BEM_E_INVALID, "bad plan or problem index");
  if (prec != BEM_C128 && prec != BEM_C64) return fail(BEM_E_INVALID, "bad precision");
  const int i = prec == BEM_C64 ? 1 : 0;
  const int nd_max = i ? P->f32.n_direct : P->f64.n_direct;
  if (schedule >= SCHED_COUNT) return fail(BEM_E_INVALID, "bad schedule");
  if (direct_depth > nd_max) return fail(BEM_E_INVALID, "direct depth beyond the one built");
  if (schedule >= 0) P->sched[i] = schedule;
  if (p2p_grid >= 0) P->p2p_cap[i] = p2p_grid;
  if (m2l_grid >= 0) P->m2l_cap[i] = m2l_grid;
  if (direct_depth >= 0) P->ndir[i] = direct_depth;
  return BEM_OK;
}

int bem_profile_start(bem_plan* plan, int prob) {
  Problem* P = get_prob(plan, prob);
  if (!P) return fail(BEM_E_INVALID, "bad plan or problem index");
  P->prof_on = true;
  P->prof_leaf = false;
  P->prof_serial = false;
  P->ev_used = 0;
  P->ev_slot.clear();
  return BEM_OK;
}

int bem_profile_serial_start(bem_plan* plan, int prob) {
  int r = bem_profile_start(plan, prob);
  if (r) return r;
  plan->probs[prob]->prof_serial = true;
  return BEM_OK;
}

int bem_profile_leaf_m2l_start(bem_plan* plan, int prob) {
  Problem* P = get_prob(plan, prob);
  if (!P) return fail(BEM_E_INVALID, "bad plan or problem index");
  // enough event pairs for a few hundred products, created outside the
  // region being timed
  while (P->ev_pool.size() < 1024) {
    hipEvent_t e;
    BEM_HIP_TRY(hipEventCreate(&e));
    P->ev_pool.push_back(e);
  }
  P->prof_on = false;
  P->prof_leaf = true;
  P->prof_serial = false;
  P->ev_used = 0;
  P->ev_slot.clear();
  return BEM_OK;
}

int bem_profile_stop(bem_plan* plan, int prob, double* ms, int32_t* calls) {
  Problem* P = get_prob(plan, prob);
  if (!P || !ms || !calls) return fail(BEM_E_INVALID, "bad arguments");
  for (int t = 0; t < PROF_SLOTS; ++t) {
    ms[t] = 0.0;
    calls[t] = 0;
  }
  for (int i = 0; i < P->ev_used; ++i) {
    BEM_HIP_TRY(hipEventSynchronize(P->ev_pool[2 * i + 1]));
    float t = 0.f;
    BEM_HIP_TRY(hipEventElapsedTime(&t, P->ev_pool[2 * i], P->ev_pool[2 * i + 1]));
    int slot = P->ev_slot[i];
    ms[slot] += t;
    calls[slot] += 1;
  }
  P->prof_on = false;
  P->prof_leaf = false;
  P->prof_serial = false;
  P->ev_used = 0;
  P->ev_slot.clear();
  return BEM_OK;
}

}  // extern "C"
