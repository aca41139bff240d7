// extern "C" entry points of the registration library (declared in include/nkreg.h).
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>

#include <algorithm>

#include "group.hpp"
#include "trace.hpp"
#include "problem.hpp"

struct nkreg_problem {
  nk::ProblemBase* impl;
};

// A batch replays one HIP graph per operation (the Hessian matvec and the objective
// and gradient). Items whose recorded launch sequences have the same shape (same
// grid, steps, scheme and precision) form a group; every launch of a group's sequence
// becomes one launch over all its items, whose per-item arguments come from a device
// table. Groups are independent branches of the graph, each captured on a branch
// stream of the batch.
// Group form value of a group that runs its sweeps in the persistent small-grid kernel.
constexpr int kFormPersistent = -2;

struct BatchGraph {
  hipGraphExec_t exec = nullptr;
  void* tables = nullptr;  // device argument tables of the captured graph
  std::vector<int> group_sizes, variants;  // per group: items, column pass (8, 0 = tiled, or kFormPersistent)
  std::vector<const void*> key_in;
  std::vector<void*> key_out;
  std::vector<unsigned> key_gen;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (tables) (void)hipFree(tables);
    exec = nullptr;
    tables = nullptr;
  }
  ~BatchGraph() { reset(); }
};

struct nkreg_batch {
  std::vector<nkreg_problem*> items;
  bool owns_items = false;  // created by nkreg_batch_create (destroyed with the batch)
  hipStream_t s = nullptr;
  std::vector<hipStream_t> branch;  // capture branches, one per group
  hipEvent_t fork = nullptr, done = nullptr;
  std::vector<hipEvent_t> joins, waits;
  BatchGraph matvec, gradient;
  std::vector<hipStream_t> lanes;       // batched PCG: streams for the items' vector work
  std::vector<hipEvent_t> lane_done;
  hipEvent_t mv_done = nullptr;
  ~nkreg_batch() {
    if (s) (void)hipStreamSynchronize(s);
    for (hipStream_t st : lanes) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
    for (hipEvent_t e : lane_done) (void)hipEventDestroy(e);
    if (mv_done) (void)hipEventDestroy(mv_done);
    matvec.reset();
    gradient.reset();
    for (hipEvent_t e : joins) (void)hipEventDestroy(e);
    for (hipEvent_t e : waits) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (done) (void)hipEventDestroy(done);
    for (hipStream_t st : branch) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
    if (s) (void)hipStreamDestroy(s);
    if (owns_items) {
      for (nkreg_problem* p : items) {
        if (!p) continue;
        (void)hipStreamSynchronize(p->impl->stream());
        delete p->impl;
        delete p;
      }
    }
  }
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

}  // namespace

namespace nk {
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace nk

namespace {

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const nk::HipError& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(NKREG_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(NKREG_EHIP, e.what());
  } catch (...) {
    return fail(NKREG_EHIP, "unknown error");
  }
}

bool pow2_in_range(int v) { return v >= nk::kMinN && v <= nk::kMaxN && (v & (v - 1)) == 0; }

int validate(const nkreg_config* c) {
  if (!c) return fail(NKREG_EINVAL, "null config");
  if (c->dim != 2 && c->dim != 3) return fail(NKREG_EINVAL, "dim must be 2 or 3");
  if (c->reg != 1 && c->reg != 2) return fail(NKREG_EINVAL, "reg must be 1 (H1) or 2 (H2)");
  if (!(c->beta > 0.0)) return fail(NKREG_EINVAL, "beta must be positive");
  if (c->nt < 1) return fail(NKREG_EINVAL, "nt must be >= 1");
  if (c->nc < 1 || c->nc > nk::kMaxNc) return fail(NKREG_EINVAL, "nc must be in [1, 16]");
  if (c->precision != 32 && c->precision != 64) return fail(NKREG_EINVAL, "precision must be 32 or 64");
  if (c->incompressible != 0 && c->incompressible != 1) return fail(NKREG_EINVAL, "incompressible must be 0 or 1");
  if (c->checkpoint_every < 0) return fail(NKREG_EINVAL, "checkpoint_every must be >= 0");
  if (c->trajectory_slots < 0) return fail(NKREG_EINVAL, "trajectory_slots must be >= 0");
  for (int i = 0; i < c->dim; ++i)
    if (!pow2_in_range(c->n[i])) return fail(NKREG_ESHAPE, "grid sizes must be powers of two in [8, 512]");
  return NKREG_OK;
}

#define NEED(ptr)                                                        \
  do {                                                                   \
    if (!(ptr)) return fail(NKREG_EINVAL, "null argument: " #ptr);       \
  } while (0)

}  // namespace

extern "C" {

const char* nkreg_version(void) { return "nkreg 1.0 gfx950"; }

const char* nkreg_status_string(int s) {
  switch (s) {
    case NKREG_OK: return "ok";
    case NKREG_EINVAL: return "invalid argument";
    case NKREG_ESHAPE: return "unsupported shape";
    case NKREG_ENOMEM: return "out of device memory";
    case NKREG_EHIP: return "HIP runtime error";
    case NKREG_ESTATE: return "call order: no cached state";
    case NKREG_ENONFINITE: return "non-finite value";
    case NKREG_ECFL: return "CFL bound violated";
    case NKREG_ENOCONV: return "iteration limit reached";
    case NKREG_ENOTIMPL: return "not implemented";
    default: return "unknown status";
  }
}

const char* nkreg_last_error(void) { return g_last_error.c_str(); }

int nkreg_create(const nkreg_config* cfg, void* hip_stream, nkreg_problem** out) {
  NEED(out);
  *out = nullptr;
  int st = validate(cfg);
  if (st != NKREG_OK) return st;
  return guarded([&]() {
    hipStream_t s = (hipStream_t)hip_stream;
    nk::ProblemBase* impl;
    impl = nk::make_problem(*cfg, s);
    *out = new nkreg_problem{impl};
    return (int)NKREG_OK;
  });
}

int nkreg_destroy(nkreg_problem* p) {
  if (!p) return NKREG_OK;
  return guarded([&]() {
    (void)hipStreamSynchronize(p->impl->stream());
    delete p->impl;
    delete p;
    return (int)NKREG_OK;
  });
}

int nkreg_set_beta(nkreg_problem* p, double beta) {
  NEED(p);
  if (!(beta > 0.0)) return fail(NKREG_EINVAL, "beta must be positive");
  return guarded([&]() { p->impl->set_beta(beta); return (int)NKREG_OK; });
}

int nkreg_use_graphs(nkreg_problem* p, int enable) {
  NEED(p);
  return guarded([&]() { p->impl->use_graph_capture(enable != 0); return (int)NKREG_OK; });
}

int nkreg_describe(nkreg_problem* p, char* buf, int len) {
  NEED(p); NEED(buf);
  if (len < 1) return fail(NKREG_EINVAL, "buffer length must be positive");
  return guarded([&]() {
    const std::string d = p->impl->describe();
    std::snprintf(buf, (size_t)len, "%s", d.c_str());
    return (int)NKREG_OK;
  });
}

int nkreg_set_images(nkreg_problem* p, const void* mT, const void* mR) {
  NEED(p); NEED(mT); NEED(mR);
  return guarded([&]() { p->impl->set_images(mT, mR); return (int)NKREG_OK; });
}

int nkreg_forward(nkreg_problem* p, const void* v, void* m1) {
  NEED(p); NEED(v);
  return guarded([&]() {
    const nk::Range range("nkreg_forward");
    p->impl->forward(v, m1);
    return (int)NKREG_OK;
  });
}

int nkreg_objective(nkreg_problem* p, const void* v, double* J, double* Jd, double* Jr) {
  NEED(p); NEED(v);
  return guarded([&]() {
    const nk::Range range("nkreg_objective");
    p->impl->objective(v, J, Jd, Jr);
    return (int)NKREG_OK;
  });
}

int nkreg_objective_gradient(nkreg_problem* p, const void* v, double* J, double* Jd, double* Jr, void* g) {
  NEED(p); NEED(v);
  return guarded([&]() {
    const nk::Range range("nkreg_objective_gradient");
    p->impl->objective_gradient(v, J, Jd, Jr, g);
    return (int)NKREG_OK;
  });
}

int nkreg_hessian_matvec(nkreg_problem* p, const void* vt, void* out) {
  NEED(p); NEED(vt); NEED(out);
  if (vt == out) return fail(NKREG_EINVAL, "input and output may not alias");
  return guarded([&]() {
    const nk::Range range("nkreg_hessian_matvec");
    p->impl->hessian_matvec(vt, out);
    return (int)NKREG_OK;
  });
}

int nkreg_precond_apply(nkreg_problem* p, const void* r, void* z) {
  NEED(p); NEED(r); NEED(z);
  return guarded([&]() {
    const nk::Range range("nkreg_precond_apply");
    p->impl->precond(r, z);
    return (int)NKREG_OK;
  });
}

int nkreg_project(nkreg_problem* p, const void* f, void* out) {
  NEED(p); NEED(f); NEED(out);
  return guarded([&]() { p->impl->project(f, out); return (int)NKREG_OK; });
}

int nkreg_pcg(nkreg_problem* p, const void* rhs, void* s, double rtol, int maxit, int* iters, double* relres) {
  NEED(p); NEED(rhs); NEED(s);
  if (!(rtol >= 0.0)) return fail(NKREG_EINVAL, "rtol must be >= 0");
  return guarded([&]() {
    const nk::Range range("nkreg_pcg");
    return p->impl->pcg(rhs, s, rtol, maxit, iters, relres);
  });
}

int nkreg_det_grad_y(nkreg_problem* p, const void* v, void* detF, double* stats) {
  NEED(p); NEED(v);
  return guarded([&]() {
    const nk::Range range("nkreg_det_grad_y");
    p->impl->det_grad_y(v, detF, stats);
    return (int)NKREG_OK;
  });
}

int nkreg_newton_solve(nkreg_problem* p, void* v, const nkreg_solve_opts* opts, nkreg_solve_report* rep) {
  NEED(p); NEED(v);
  return guarded([&]() {
    const nk::Range range("nkreg_newton_solve");
    return p->impl->newton(v, opts, rep);
  });
}

int nkreg_picard_solve(nkreg_problem* p, void* v, const nkreg_solve_opts* opts, const nkreg_picard_opts* popts,
                       nkreg_solve_report* rep) {
  NEED(p); NEED(v);
  return guarded([&]() {
    const nk::Range range("nkreg_picard_solve");
    return p->impl->picard(v, opts, popts, rep);
  });
}

int nkreg_hessian_lanczos(nkreg_problem* p, int steps, double* ritz, int* count) {
  NEED(p); NEED(ritz);
  return guarded([&]() {
    const nk::Range range("nkreg_hessian_lanczos");
    return p->impl->lanczos(steps, ritz, count);
  });
}

int nkreg_set_hessian(nkreg_problem* p, int mode) {
  NEED(p);
  return guarded([&]() { p->impl->set_hessian(mode); return (int)NKREG_OK; });
}

int nkreg_continuation(nkreg_problem* p, void* v, const double* betas, int levels, const nkreg_solve_opts* opts,
                       nkreg_solve_report* reports) {
  NEED(p); NEED(v);
  if (levels < 0 || (levels > 0 && !betas)) return fail(NKREG_EINVAL, "bad beta levels");
  return guarded([&]() {
    const nk::Range range("nkreg_continuation");
    return p->impl->continuation(v, betas, levels, opts, reports);
  });
}

int nkreg_beta_search(nkreg_problem* p, void* v, const nkreg_beta_search_opts* opts, nkreg_beta_search_report* rep) {
  NEED(p); NEED(v); NEED(opts);
  return guarded([&]() {
    const nk::Range range("nkreg_beta_search");
    return p->impl->beta_search(v, opts, rep);
  });
}

int nkreg_gradient(nkreg_problem* p, const void* u, void* g) {
  NEED(p); NEED(u); NEED(g);
  return guarded([&]() { p->impl->gradient(u, g); return (int)NKREG_OK; });
}

int nkreg_divergence(nkreg_problem* p, const void* w, void* s) {
  NEED(p); NEED(w); NEED(s);
  return guarded([&]() { p->impl->divergence(w, s); return (int)NKREG_OK; });
}

int nkreg_apply_reg(nkreg_problem* p, const void* x, void* out) {
  NEED(p); NEED(x); NEED(out);
  return guarded([&]() { p->impl->apply_reg(x, out); return (int)NKREG_OK; });
}

int nkreg_dot(nkreg_problem* p, const void* a, const void* b, long long cnt, double* out) {
  NEED(p); NEED(a); NEED(b); NEED(out);
  if (cnt < 0) return fail(NKREG_EINVAL, "negative count");
  return guarded([&]() { *out = p->impl->dot(a, b, cnt); return (int)NKREG_OK; });
}

int nkreg_timer_arm(nkreg_problem* p, int kernel_id, int capacity) {
  NEED(p);
  if (capacity < 1 || capacity > (1 << 16)) return fail(NKREG_EINVAL, "capacity must be in [1, 65536]");
  return guarded([&]() { p->impl->timer_arm(kernel_id, capacity); return (int)NKREG_OK; });
}

int nkreg_matvec_bytes(nkreg_problem* p, const void* vt, void* out, double* bytes, int* launches) {
  NEED(p); NEED(vt); NEED(out);
  return guarded([&]() { p->impl->matvec_bytes(vt, out, bytes, launches); return (int)NKREG_OK; });
}

int nkreg_timer_read(nkreg_problem* p, int* launches, double* avg_ms, double* bytes_per_launch) {
  NEED(p);
  return guarded([&]() { p->impl->timer_read(launches, avg_ms, bytes_per_launch); return (int)NKREG_OK; });
}

}  // extern "C"

namespace {

// The batch's own stream and events for count items.
void batch_init(nkreg_batch* b, int count) {
  NK_HIP(hipStreamCreateWithFlags(&b->s, hipStreamNonBlocking));  // default priority
  NK_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  NK_HIP(hipEventCreateWithFlags(&b->done, hipEventDisableTiming));
  b->joins.resize(count);
  b->waits.resize(count);
  for (int i = 0; i < count; ++i) {
    NK_HIP(hipEventCreateWithFlags(&b->joins[i], hipEventDisableTiming));
    NK_HIP(hipEventCreateWithFlags(&b->waits[i], hipEventDisableTiming));
  }
}

}  // namespace

extern "C" {

int nkreg_batch_create(int count, const nkreg_config* cfgs, void* hip_stream, nkreg_batch** out) {
  NEED(out);
  *out = nullptr;
  if (count < 0 || (count > 0 && !cfgs)) return fail(NKREG_EINVAL, "bad batch");
  for (int i = 0; i < count; ++i) {
    const int st = validate(cfgs + i);
    if (st != NKREG_OK) return st;
  }
  return guarded([&]() {
    std::unique_ptr<nkreg_batch> b(new nkreg_batch);
    b->owns_items = true;
    b->items.reserve(count);
    for (int i = 0; i < count; ++i) {
      std::unique_ptr<nk::ProblemBase> impl(nk::make_problem(cfgs[i], (hipStream_t)hip_stream));
      b->items.push_back(new nkreg_problem{impl.get()});
      impl.release();
    }
    batch_init(b.get(), count);
    *out = b.release();
    return (int)NKREG_OK;
  });
}

int nkreg_batch_wrap(int count, nkreg_problem* const* items, nkreg_batch** out) {
  NEED(out);
  *out = nullptr;
  if (count < 0 || (count > 0 && !items)) return fail(NKREG_EINVAL, "bad batch");
  for (int i = 0; i < count; ++i)
    if (!items[i]) return fail(NKREG_EINVAL, "null batch item");
  return guarded([&]() {
    std::unique_ptr<nkreg_batch> b(new nkreg_batch);
    b->items.assign(items, items + count);
    batch_init(b.get(), count);
    *out = b.release();
    return (int)NKREG_OK;
  });
}

int nkreg_batch_item(nkreg_batch* b, int i, nkreg_problem** out) {
  NEED(b); NEED(out);
  if (i < 0 || i >= (int)b->items.size()) return fail(NKREG_EINVAL, "batch item index out of range");
  *out = b->items[i];
  return NKREG_OK;
}

int nkreg_batch_destroy(nkreg_batch* b) {
  delete b;
  return NKREG_OK;
}

}  // extern "C"

namespace {

using nk::add_tables;
using nk::capture_group;
using nk::GroupPlan;
using nk::issue_group;
using nk::same_sequence;
using nk::time_group;

// Joins groups whose sequences differ only in their time loops' iteration counts
// (items with different step counts and no checkpointing) into one group each; the
// joined group's sequences are padded with inactive launches (group.hpp).
std::vector<GroupPlan> merge_ragged(nkreg_batch* b, std::vector<GroupPlan> plans) {
  auto eligible = [&](const GroupPlan& gp) { return b->items[gp.items[0]]->impl->cfg.checkpoint_every == 0; };
  std::vector<std::vector<size_t>> clusters;
  for (size_t i = 0; i < plans.size(); ++i) {
    bool placed = false;
    if (eligible(plans[i])) {
      for (auto& c : clusters) {
        bool ok = eligible(plans[c[0]]);
        for (size_t k = 0; ok && k < c.size(); ++k) ok = nk::ragged_compatible(plans[c[k]].recs[0], plans[i].recs[0]);
        if (ok) {
          c.push_back(i);
          placed = true;
          break;
        }
      }
    }
    if (!placed) clusters.push_back({i});
  }
  std::vector<GroupPlan> out;
  for (const auto& c : clusters) {
    if (c.size() == 1) {
      out.push_back(std::move(plans[c[0]]));
      continue;
    }
    GroupPlan m;
    m.ragged = true;
    std::vector<nk::Recorder> all;
    for (size_t i : c)
      for (size_t k = 0; k < plans[i].items.size(); ++k) {
        m.items.push_back(plans[i].items[k]);
        all.push_back(std::move(plans[i].recs[k]));
      }
    m.recs = nk::pad_ragged(all);
    for (const auto& r : m.recs)
      if (!same_sequence(m.recs[0].recs, r.recs)) throw nk::HipError(NKREG_EHIP, "padded group sequences differ");
    out.push_back(std::move(m));
  }
  return out;
}

// Records an item's launch sequence for one batched operation (column pass variant
// cv >= 0 overrides the item's own choice).
using RecordFn = void (*)(nk::ProblemBase*, const void*, void*, nk::Recorder&, int);

void record_matvec_fn(nk::ProblemBase* p, const void* in, void* out, nk::Recorder& r, int cv) {
  p->record_matvec(in, out, r, cv);
}
void record_gradient_fn(nk::ProblemBase* p, const void* in, void* out, nk::Recorder& r, int cv) {
  p->record_gradient(in, out, r, cv);
}

// One batched operation: (re)builds the batch graph bg of the operation when the
// pointer sets or an item's configuration changed, then replays it, ordered after
// every earlier call on the items' streams.
void run_batch(nkreg_batch* b, BatchGraph& bg, RecordFn record, const void* const* vt, void* const* out) {
  {
    const size_t cnt = b->items.size();
    if (cnt == 0) return;
    // items on one caller stream: the graph replays on that stream, ordered like
    // any other call; otherwise on the batch stream, joined to every caller stream
    const hipStream_t cs = b->items[0]->impl->caller_stream();
    bool one_stream = true;
    for (size_t i = 1; i < cnt; ++i) one_stream = one_stream && b->items[i]->impl->caller_stream() == cs;
    bool stale = !bg.exec || bg.key_in.size() != cnt;
    for (size_t i = 0; i < cnt && !stale; ++i)
      stale = bg.key_in[i] != vt[i] || bg.key_out[i] != out[i] || bg.key_gen[i] != b->items[i]->impl->generation;
    if (stale || !one_stream) {
      // the batch stream waits for every caller stream (and so for all earlier
      // work on the items), also before a rebuild replays a group to time it
      for (size_t i = 0; i < cnt; ++i) {
        NK_HIP(hipEventRecord(b->waits[i], b->items[i]->impl->caller_stream()));
        NK_HIP(hipStreamWaitEvent(b->s, b->waits[i], 0));
      }
    }
    if (stale) {
      NK_HIP(hipStreamSynchronize(b->s));
      bg.reset();
      // record every item's matvec and group equal-shaped sequences
      std::vector<nk::Recorder> recs(cnt);
      for (size_t i = 0; i < cnt; ++i) record(b->items[i]->impl, vt[i], out[i], recs[i], -1);
      std::vector<GroupPlan> plans;
      for (size_t i = 0; i < cnt; ++i) {
        bool placed = false;
        for (auto& gp : plans) {
          if (same_sequence(gp.recs[0].recs, recs[i].recs)) {
            gp.items.push_back(i);
            gp.recs.push_back(std::move(recs[i]));
            placed = true;
            break;
          }
        }
        if (!placed) {
          plans.emplace_back();
          plans.back().items.push_back(i);
          plans.back().recs.push_back(std::move(recs[i]));
        }
      }
      if (nk::ragged_enabled()) plans = merge_ragged(b, std::move(plans));
      // an item group's sequences recorded with column variant cv (padded to the
      // group's longest loops for a group of several step counts)
      auto record_plan = [&](const GroupPlan& gp, int cv) {
        GroupPlan c;
        c.items = gp.items;
        c.ragged = gp.ragged;
        c.recs.resize(gp.items.size());
        for (size_t k = 0; k < gp.items.size(); ++k)
          record(b->items[gp.items[k]]->impl, vt[gp.items[k]], out[gp.items[k]], c.recs[k], cv);
        if (c.ragged) c.recs = nk::pad_ragged(c.recs);
        return c;
      };
      // Small square grids run their sweeps in the persistent kernel (recorded with the
      // 8-per-lane column pass it runs; the values are those of any column pass).
      // Otherwise a group's launches are G times larger than one item's: where the
      // tiled column pass applies, time both column passes (identical values) at the
      // group's scale and keep the faster.
      bg.variants.clear();
      for (auto& gp : plans) {
        nk::ProblemBase* first = b->items[gp.items[0]]->impl;
        int chosen = first->col_variant();
        if (nk::small_config(first->cfg)) {
          GroupPlan c = record_plan(gp, 8);
          c.small_ops = nk::small_prefix(c.recs[0].recs);
          if (c.small_ops) {
            // the persistent form against plain launches, timed at the group's scale
            std::vector<GroupPlan> cands(2, c);
            cands[1].small_ops = 0;
            const size_t pick = nk::fastest_plan(cands, b->s);
            gp = std::move(cands[pick]);
            bg.variants.push_back(gp.small_ops ? kFormPersistent : 8);
            continue;
          }
        }
        if (gp.items.size() > 1 && first->tiled_pass_applies() && (chosen == 8 || chosen == 0)) {
          float best = 0.f;
          GroupPlan bestp;
          for (int cv : {8, 0}) {
            GroupPlan c = record_plan(gp, cv);
            const float ms = time_group(c, b->s);
            if (cv == 8 || ms < best) { best = ms; bestp = std::move(c); chosen = cv; }
          }
          gp = std::move(bestp);
        }
        bg.variants.push_back(chosen);
      }
      std::vector<unsigned char> host;
      for (auto& gp : plans) add_tables(gp, host);
      if (!host.empty()) {
        NK_HIP(hipMalloc(&bg.tables, host.size()));
        NK_HIP(hipMemcpy(bg.tables, host.data(), host.size(), hipMemcpyHostToDevice));
      }
      bg.group_sizes.clear();
      for (auto& gp : plans) bg.group_sizes.push_back((int)gp.items.size());
      // groups become parallel branches of the graph: each is captured on a
      // stream of its own, forked from and joined back into the batch stream
      while (b->branch.size() < plans.size()) {
        hipStream_t st = nullptr;
        NK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));  // default priority
        b->branch.push_back(st);
      }
      hipGraph_t graph = nullptr;
      NK_HIP(hipStreamBeginCapture(b->s, hipStreamCaptureModeThreadLocal));
      try {
        NK_HIP(hipEventRecord(b->fork, b->s));
        for (size_t gi = 0; gi < plans.size(); ++gi) {
          hipStream_t st = b->branch[gi];
          NK_HIP(hipStreamWaitEvent(st, b->fork, 0));
          issue_group(plans[gi], bg.tables, st);
          NK_HIP(hipEventRecord(b->joins[gi], st));
          NK_HIP(hipStreamWaitEvent(b->s, b->joins[gi], 0));
        }
      } catch (...) {
        (void)hipStreamEndCapture(b->s, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
      }
      NK_HIP(hipStreamEndCapture(b->s, &graph));
      const hipError_t e = hipGraphInstantiate(&bg.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) {
        bg.exec = nullptr;
        throw nk::HipError(NKREG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      }
      bg.key_in.assign(vt, vt + cnt);
      bg.key_out.assign(out, out + cnt);
      bg.key_gen.resize(cnt);
      for (size_t i = 0; i < cnt; ++i) bg.key_gen[i] = b->items[i]->impl->generation;
    }
    if (one_stream) {
      NK_HIP(hipGraphLaunch(bg.exec, cs));
      return;
    }
    // every caller stream waits for the batch
    NK_HIP(hipGraphLaunch(bg.exec, b->s));
    NK_HIP(hipEventRecord(b->done, b->s));
    for (size_t i = 0; i < cnt; ++i) NK_HIP(hipStreamWaitEvent(b->items[i]->impl->caller_stream(), b->done, 0));
  }
}


// Columns of the dense Hessian assembled per graph replay: up to this many, and
// fewer on large grids, where one matvec already fills the GPU.
constexpr int kAssembleGroup = 32;

// Dense Hessian by unit-vector matvecs, G columns per replay. The handle and G - 1
// clones of it (same configuration, images, velocity and Hessian mode, so every
// clone's matvec is bit-identical to the handle's) form one batch group whose
// launch sequence is captured once; each replay takes G unit vectors and yields
// G adjacent columns of H (column-major, nv x nv).
void assemble_grouped(nk::ProblemBase* src, double* H) {
  if (!src->state_ready()) throw nk::HipError(NKREG_ESTATE, "no gradient computed at the current velocity");
  const nkreg_config c = src->cfg;
  const long long npts = (long long)c.n[0] * c.n[1] * (c.dim == 3 ? c.n[2] : 1);
  const long long nv = (long long)c.nc * c.dim * npts;
  const int G = (int)std::min<long long>(std::min<long long>(kAssembleGroup, nv),
                                         std::max<long long>(1, (1LL << 20) / npts));
  if (G <= 1) {
    src->assemble_hessian(H);
    return;
  }
  const hipStream_t st = src->stream();
  std::vector<std::unique_ptr<nk::ProblemBase>> clones;
  std::vector<nk::ProblemBase*> items{src};
  const void *mT = nullptr, *mR = nullptr;
  src->images(&mT, &mR);
  for (int i = 1; i < G; ++i) {
    nk::ProblemBase* q = nk::make_problem(c, st);
    clones.emplace_back(q);
    q->set_hessian(src->hessian_mode());
    q->set_centred_images(mT, mR, src->image_shift());
    q->objective_gradient(src->velocity(), nullptr, nullptr, nullptr, nullptr);
    items.push_back(q);
  }
  nk::DevBuf<double> E((size_t)G * nv), C((size_t)G * nv);
  GroupPlan gp;
  gp.recs.resize(G);
  const int cv = nk::small_config(c) ? 8 : -1;
  for (int i = 0; i < G; ++i) {
    gp.items.push_back((size_t)i);
    items[i]->record_matvec(E.p + (size_t)i * nv, C.p + (size_t)i * nv, gp.recs[i], cv);
    if (!same_sequence(gp.recs[0].recs, gp.recs[i].recs))
      throw nk::HipError(NKREG_EHIP, "clone's matvec differs from the handle's");
  }
  gp.small_ops = cv == 8 ? nk::small_prefix(gp.recs[0].recs) : 0;
  if (gp.small_ops) {
    // the persistent form against plain launches, timed at the group's scale
    std::vector<GroupPlan> cands(2, gp);
    cands[1].small_ops = 0;
    NK_HIP(hipStreamSynchronize(st));
    hipStream_t tst = nullptr;
    NK_HIP(hipStreamCreateWithFlags(&tst, hipStreamNonBlocking));  // default priority
    size_t pick = 0;
    std::vector<float> ms;
    try {
      pick = nk::fastest_plan(cands, tst, &ms);
    } catch (...) {
      (void)hipStreamDestroy(tst);
      throw;
    }
    (void)hipStreamDestroy(tst);
    gp = std::move(cands[pick]);
    src->assembly_timing = std::to_string(G) + " columns per replay: persistent " + std::to_string(1e3f * ms[0]) +
                           " us, launches " + std::to_string(1e3f * ms[1]) + " us; chose " +
                           (gp.small_ops ? "persistent" : "launches");
  }
  std::vector<unsigned char> host;
  add_tables(gp, host);
  nk::DevBuf<unsigned char> tab(host.size());
  if (!host.empty()) NK_HIP(hipMemcpy(tab.p, host.data(), host.size(), hipMemcpyHostToDevice));
  // captured on a stream of its own (the caller's may be the null stream), replayed on st
  hipStream_t cap = nullptr;
  NK_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));  // default priority
  hipGraphExec_t ex = nullptr;
  try {
    ex = capture_group(gp, tab.p, cap);
  } catch (...) {
    (void)hipStreamDestroy(cap);
    throw;
  }
  (void)hipStreamDestroy(cap);
  try {
    const long long tot = (long long)G * nv;
    const int blocks = (int)std::min<long long>((tot + 255) / 256, 8192);
    for (long long j0 = 0; j0 < nv; j0 += G) {
      hipLaunchKernelGGL(nk::k_unit_block, dim3(blocks), dim3(256), 0, st, nv, G, j0, E.p);
      NK_LAUNCHED();
      NK_HIP(hipGraphLaunch(ex, st));
      const long long cols = std::min<long long>(G, nv - j0);
      NK_HIP(hipMemcpyAsync(H + (size_t)j0 * nv, C.p, (size_t)cols * nv * sizeof(double), hipMemcpyDeviceToDevice,
                            st));
    }
    NK_HIP(hipStreamSynchronize(st));
  } catch (...) {
    (void)hipStreamSynchronize(st);
    (void)hipGraphExecDestroy(ex);
    throw;
  }
  (void)hipGraphExecDestroy(ex);
}

}  // namespace

extern "C" {

int nkreg_hessian_assemble(nkreg_problem* p, void* H) {
  NEED(p); NEED(H);
  return guarded([&]() {
    const nk::Range range("nkreg_hessian_assemble");
    assemble_grouped(p->impl, (double*)H); return (int)NKREG_OK;
  });
}

int nkreg_batch_hessian_matvec(nkreg_batch* b, const void* const* vt, void* const* out) {
  NEED(b);
  if (!b->items.empty()) { NEED(vt); NEED(out); }
  for (size_t i = 0; i < b->items.size(); ++i)
    if (!vt[i] || !out[i] || vt[i] == out[i]) return fail(NKREG_EINVAL, "batch matvec: null or aliased item vectors");
  return guarded([&]() {
    const nk::Range range("nkreg_batch_hessian_matvec");
    run_batch(b, b->matvec, record_matvec_fn, vt, out);
    return (int)NKREG_OK;
  });
}

int nkreg_batch_objective_gradient(nkreg_batch* b, const void* const* v, double* J, double* J_dist, double* J_reg,
                                   void* const* g) {
  NEED(b);
  if (!b->items.empty()) NEED(v);
  for (size_t i = 0; i < b->items.size(); ++i)
    if (!v[i]) return fail(NKREG_EINVAL, "batch gradient: null velocity");
  return guarded([&]() {
    const nk::Range range("nkreg_batch_objective_gradient");
    const size_t cnt = b->items.size();
    for (size_t i = 0; i < cnt; ++i) b->items[i]->impl->check_cfl(v[i]);
    std::vector<void*> gout(cnt, nullptr);
    if (g)
      for (size_t i = 0; i < cnt; ++i) gout[i] = g[i];
    run_batch(b, b->gradient, record_gradient_fn, v, gout.data());
    for (size_t i = 0; i < cnt; ++i)
      b->items[i]->impl->gradient_done(J ? J + i : nullptr, J_dist ? J_dist + i : nullptr,
                                       J_reg ? J_reg + i : nullptr);
    return (int)NKREG_OK;
  });
}

int nkreg_batch_pcg(nkreg_batch* b, const void* const* rhs, void* const* x, double rtol, int maxit, int* iters,
                    double* relres) {
  NEED(b);
  if (!b->items.empty()) { NEED(rhs); NEED(x); }
  if (!(rtol >= 0.0)) return fail(NKREG_EINVAL, "rtol must be >= 0");
  for (size_t i = 0; i < b->items.size(); ++i)
    if (!rhs[i] || !x[i]) return fail(NKREG_EINVAL, "batch PCG: null item vectors");
  return guarded([&]() {
    const nk::Range range("nkreg_batch_pcg");
    const size_t cnt = b->items.size();
    for (size_t i = 0; i < cnt; ++i)
      if (!b->items[i]->impl->state_ready()) throw nk::HipError(NKREG_ESTATE, "batch PCG: an item has no state");
    std::vector<const void*> ps(cnt);
    std::vector<void*> qs(cnt);
    bool any = false;
    for (size_t i = 0; i < cnt; ++i) {
      nk::ProblemBase* p = b->items[i]->impl;
      any = p->pcg_begin(rhs[i], x[i], rtol, maxit) || any;
      ps[i] = p->pcg_p();
      qs[i] = p->pcg_q();
    }
    // Every iteration: one batched matvec for all items (an item that has stopped keeps its
    // direction, so its product is recomputed unchanged and unused), then each active
    // item's own vector work, spread over a few streams so that the items' small launches
    // overlap, and one wait for all of them. The streams only reorder independent items'
    // work: every item runs the kernels of its own PCG in its own order.
    const size_t nl = std::min<size_t>(cnt, 8);
    while (b->lanes.size() < nl) {
      hipStream_t st = nullptr;
      NK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));  // default priority
      b->lanes.push_back(st);
    }
    while (b->lane_done.size() < nl) {
      hipEvent_t e = nullptr;
      NK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b->lane_done.push_back(e);
    }
    if (!b->mv_done) NK_HIP(hipEventCreateWithFlags(&b->mv_done, hipEventDisableTiming));
    std::vector<hipStream_t> callers;
    for (size_t i = 0; i < cnt; ++i) {
      const hipStream_t cs = b->items[i]->impl->caller_stream();
      if (std::find(callers.begin(), callers.end(), cs) == callers.end()) callers.push_back(cs);
    }
    // on every way out (an error included) the items launch on their own streams again and
    // no work of theirs is left on the batch's streams
    struct Unroute {
      nkreg_batch* b;
      ~Unroute() {
        for (hipStream_t st : b->lanes) (void)hipStreamSynchronize(st);
        for (nkreg_problem* p : b->items) p->impl->route_launches(nullptr);
      }
    } unroute{b};
    int round = 0;
    while (any) {
      const nk::Range iter("batch pcg iteration", round++);
      for (nkreg_problem* p : b->items) p->impl->route_launches(nullptr);
      run_batch(b, b->matvec, record_matvec_fn, ps.data(), qs.data());
      // the streams take up the items' work after the batched matvec and after all
      // earlier work on the callers' streams
      for (hipStream_t cs : callers) {
        NK_HIP(hipEventRecord(b->mv_done, cs));
        for (size_t k = 0; k < nl; ++k) NK_HIP(hipStreamWaitEvent(b->lanes[k], b->mv_done, 0));
      }
      for (size_t i = 0; i < cnt; ++i) {
        nk::ProblemBase* p = b->items[i]->impl;
        if (!p->pcg_active()) continue;
        p->route_launches(b->lanes[i % nl]);   // pcg_finish's launches follow on the same stream
        p->pcg_step_on(b->lanes[i % nl]);
      }
      for (size_t k = 0; k < nl; ++k) NK_HIP(hipStreamSynchronize(b->lanes[k]));
      any = false;
      for (size_t i = 0; i < cnt; ++i) {
        nk::ProblemBase* p = b->items[i]->impl;
        if (!p->pcg_active()) continue;
        p->pcg_finish();
        any = p->pcg_active() || any;
      }
      // the next batched matvec (and anything after the call) waits for the items' updates
      for (size_t k = 0; k < nl; ++k) {
        NK_HIP(hipEventRecord(b->lane_done[k], b->lanes[k]));
        for (hipStream_t cs : callers) NK_HIP(hipStreamWaitEvent(cs, b->lane_done[k], 0));
      }
    }
    int status = NKREG_OK;
    for (size_t i = 0; i < cnt; ++i)
      if (b->items[i]->impl->pcg_result(iters ? iters + i : nullptr, relres ? relres + i : nullptr) != NKREG_OK)
        status = NKREG_ENOCONV;
    return status;
  });
}

int nkreg_batch_set_state(nkreg_batch* b, const void* const* v) {
  return nkreg_batch_objective_gradient(b, v, nullptr, nullptr, nullptr, nullptr);
}

int nkreg_batch_groups(nkreg_batch* b, int* groups, int* sizes, int* form, int cap) {
  NEED(b); NEED(groups);
  const BatchGraph& bg = b->matvec;
  *groups = (int)bg.group_sizes.size();
  for (int i = 0; i < cap && i < (int)bg.group_sizes.size(); ++i) {
    if (sizes) sizes[i] = bg.group_sizes[i];
    if (form) form[i] = bg.variants[i] == kFormPersistent ? 2 : bg.variants[i] == 0 ? 1 : 0;
  }
  return NKREG_OK;
}

}  // extern "C"
