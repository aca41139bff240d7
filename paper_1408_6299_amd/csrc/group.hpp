// Batch groups: the recorded launch sequences of items with equal shapes, issued as one
// launch per position over the whole group (per-item arguments from a device table), or,
// for small grids, with the leading transport launches run by one persistent kernel.
#pragma once

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/nkreg.h"
#include "small.hpp"

namespace nk {

// Whether the persistent small-grid kernel may be used: NKREG_SMALL=0 turns it off,
// NKREG_SMALL=1 forces it wherever it applies (no timing against plain launches).
inline bool small_enabled() {
  const char* e = std::getenv("NKREG_SMALL");
  return !(e && e[0] == '0');
}
inline bool small_forced() {
  const char* e = std::getenv("NKREG_SMALL");
  return e && e[0] == '1';
}

// Configurations whose matvec may run its sweeps in the persistent kernel: square 2D
// grids of at most kSmallMaxN points per axis.
inline bool small_config(const nkreg_config& c) {
  return small_enabled() && c.dim == 2 && c.n[0] == c.n[1] && c.n[0] <= kSmallMaxN;
}

// The first row stage of a sequence (its precision, row length and velocity form).
inline const LaunchRec& first_row(const std::vector<LaunchRec>& seq) {
  for (const auto& r : seq)
    if (r.kind == LaunchRec::ROW) return r;
  throw HipError(-4, "sequence without a row stage");
}
// Axis length of the sequence's column passes (0 if none).
inline int small_n1(const std::vector<LaunchRec>& seq) {
  for (const auto& r : seq)
    if (r.kind == LaunchRec::COL) return r.len;
  return 0;
}

// Leading launches of a recorded sequence that the persistent kernel runs: transport row
// stages, 8-per-lane column derivative passes, fills and FP64-to-transport conversions,
// all of one precision, on a square 2D grid of at most kSmallMaxN points per axis. Zero
// when fewer than 8 qualify.
inline size_t small_prefix(const std::vector<LaunchRec>& seq) {
  if (!small_enabled()) return 0;
  const LaunchRec* r0 = nullptr;
  for (const auto& r : seq)
    if (r.kind == LaunchRec::ROW) { r0 = &r; break; }
  const int n1 = small_n1(seq);
  if (!r0 || r0->dim != 2 || r0->len != n1 || n1 < 8 || n1 > kSmallMaxN) return 0;
  const bool f64 = r0->f64;
  size_t p = 0;
  for (; p < seq.size(); ++p) {
    const LaunchRec& r = seq[p];
    bool ok = false;
    if (r.kind == LaunchRec::ROW)
      ok = r.f64 == f64 && r.dim == 2 && r.len == n1 && r.nc1 == r0->nc1 && r.tw == r0->tw &&
           (r.stage == ST_INC1 || r.stage == ST_INC2 || r.stage == ST_ADJINIT || r.stage == ST_ADJ1 ||
            r.stage == ST_ADJ2);
    else if (r.kind == LaunchRec::COL)
      ok = r.f64 == f64 && r.stage == COL_DERIV && r.elems == 8 && r.len == n1 && r.tw == r0->tw;
    else if (r.kind == LaunchRec::FILL)
      ok = r.f64 == f64;
    else if (r.kind == LaunchRec::CONV)
      ok = !f64 && r.conv == 1;
    if (!ok) break;
  }
  return p >= 8 ? p : 0;
}

// The persistent kernel's program for the first n launches (table offsets offs).
inline std::vector<SmallOp> small_program(const std::vector<LaunchRec>& seq, const std::vector<size_t>& offs,
                                          size_t n) {
  std::vector<SmallOp> prog(n);
  for (size_t p = 0; p < n; ++p) {
    const LaunchRec& r = seq[p];
    SmallOp& o = prog[p];
    o = SmallOp{};
    o.off = (long long)offs[p];
    o.esize = (int)r.entry.size();
    o.gx = (int)r.grid.x;
    o.gy = (int)r.grid.y;
    o.gz = (int)r.grid.z;
    switch (r.kind) {
      case LaunchRec::ROW: o.kind = SOP_ROW; o.sub = r.stage; break;
      case LaunchRec::COL: o.kind = SOP_COL; o.sub = r.stage; o.ca = r.ca; o.scale = r.scale; o.twb = r.iarg; break;
      case LaunchRec::FILL: o.kind = SOP_FILL; o.scale = r.fval; o.cnt = r.cnt; break;
      default: o.kind = SOP_CONV; o.cnt = r.cnt; break;
    }
  }
  return prog;
}

// Issues one recorded launch position for a whole group (tab = its table).
inline void launch_group(const LaunchRec& r, int G, void* tab, hipStream_t st) {
  dim3 grid = r.grid;
  const unsigned z = grid.z;
  grid.z = z * (unsigned)G;
  const void* tw = r.tw;
  int iarg = r.iarg, nfz = r.nfz, inner = r.ca.inner;
  long long cnt = r.cnt;
  ColArgs ca = r.ca;
  float sf = (float)r.scale, vf = (float)r.fval;
  double sd = r.scale, vd = r.fval;
  void* args[6];
  switch (r.kind) {
    case LaunchRec::ROW: args[0] = &tab; args[1] = &tw; args[2] = &iarg; break;
    case LaunchRec::COL:
      args[0] = &tab; args[1] = &ca; args[2] = r.f64 ? (void*)&sd : (void*)&sf; args[3] = &tw; args[4] = &iarg;
      args[5] = &nfz;
      break;
    case LaunchRec::FILL: args[0] = &cnt; args[1] = r.f64 ? (void*)&vd : (void*)&vf; args[2] = &tab; break;
    case LaunchRec::CONV: args[0] = &cnt; args[1] = &tab; break;
    case LaunchRec::SPEC: args[0] = &tab; args[1] = &iarg; break;
    case LaunchRec::SPECCOL: args[0] = &tab; args[1] = &inner; args[2] = &tw; args[3] = &iarg; break;
    case LaunchRec::RED: args[0] = &cnt; args[1] = &tab; break;
    case LaunchRec::REDF: args[0] = &iarg; args[1] = &tab; break;
    default: throw HipError(NKREG_EHIP, "unexpected recorded launch");
  }
  NK_HIP(hipLaunchKernel(r.kernel, grid, r.block, args, 0, st));
}

inline bool same_sequence(const std::vector<LaunchRec>& a, const std::vector<LaunchRec>& b) {
  if (a.size() != b.size()) return false;
  for (size_t i = 0; i < a.size(); ++i)
    if (!a[i].same_shape(b[i])) return false;
  return true;
}

// ---- items with different step counts in one group ----
// Items whose operations differ only in their number of time steps record the same
// launches outside the time loops and the same launches in each loop iteration they
// share. Such items form one group: an item whose loop has ended rides along with
// the others' remaining iterations as an inactive table entry, which the group
// kernels skip. Every item still runs exactly its own launches, so its results are
// those of its own operation. NKREG_RAGGED=0 keeps one group per step count.
inline bool ragged_enabled() {
  const char* e = std::getenv("NKREG_RAGGED");
  return !(e && e[0] == '0');
}

// A recorded sequence cut at its time-loop marks: runs outside every loop (loop 0,
// one range) and time loops (one range per iteration). Ranges are [first, last).
struct SeqBlock {
  int loop = 0;
  std::vector<std::pair<size_t, size_t>> ranges;
};
// Returns false (and no blocks) when the marks do not describe whole loops in order,
// as in a checkpointed sweep, whose segment recomputations nest inside the adjoint loop.
inline bool cut_sequence(const Recorder& r, std::vector<SeqBlock>& out) {
  out.clear();
  struct Piece { size_t a, b; int loop, step; };
  std::vector<Piece> pieces;
  size_t pos = 0;
  int loop = 0, step = 0;
  for (const auto& m : r.marks) {
    if (m.pos > pos) pieces.push_back({pos, m.pos, loop, step});
    pos = m.pos > pos ? m.pos : pos;
    loop = m.loop;
    step = m.step;
  }
  if (r.recs.size() > pos) pieces.push_back({pos, r.recs.size(), loop, step});
  for (const auto& p : pieces) {
    if (p.loop == 0) {
      if (!out.empty() && out.back().loop == 0) out.back().ranges.back().second = p.b;
      else out.push_back({0, {{p.a, p.b}}});
    } else if (!out.empty() && out.back().loop == p.loop && p.step == (int)out.back().ranges.size()) {
      out.back().ranges.push_back({p.a, p.b});
    } else if (p.step == 0) {
      out.push_back({p.loop, {{p.a, p.b}}});
    } else {
      out.clear();
      return false;
    }
  }
  return true;
}

inline bool same_range(const std::vector<LaunchRec>& a, std::pair<size_t, size_t> ra, const std::vector<LaunchRec>& b,
                       std::pair<size_t, size_t> rb, bool loop) {
  if (ra.second - ra.first != rb.second - rb.first) return false;
  for (size_t k = 0; k < ra.second - ra.first; ++k) {
    const LaunchRec& x = a[ra.first + k];
    if (!x.same_shape(b[rb.first + k])) return false;
    if (loop && x.kind != LaunchRec::ROW && x.kind != LaunchRec::COL) return false;
  }
  return true;
}

// True if two recorded sequences differ at most in their time loops' iteration counts
// (and then only in launches the group kernels can skip).
inline bool ragged_compatible(const Recorder& a, const Recorder& b) {
  std::vector<SeqBlock> ca, cb;
  if (!cut_sequence(a, ca) || !cut_sequence(b, cb) || ca.size() != cb.size()) return false;
  for (size_t i = 0; i < ca.size(); ++i) {
    if (ca[i].loop != cb[i].loop) return false;
    if (ca[i].loop == 0) {
      if (!same_range(a.recs, ca[i].ranges[0], b.recs, cb[i].ranges[0], false)) return false;
      continue;
    }
    const size_t n = std::min(ca[i].ranges.size(), cb[i].ranges.size());
    for (size_t s = 0; s < n; ++s)
      if (!same_range(a.recs, ca[i].ranges[s], b.recs, cb[i].ranges[s], true)) return false;
  }
  return true;
}

// A copy of a recorded row stage or column pass whose table entry is marked inactive.
inline LaunchRec inactive_copy(const LaunchRec& r) {
  LaunchRec c = r;
  auto flag = [&](auto proto) {
    using T = decltype(proto);
    if (c.entry.size() != sizeof(T)) throw HipError(NKREG_EHIP, "unexpected table entry size");
    T v;
    std::memcpy(&v, c.entry.data(), sizeof(T));
    v.inactive = 1;
    std::memcpy(c.entry.data(), &v, sizeof(T));
  };
  if (r.kind == LaunchRec::ROW) {
    if (r.f64) flag(StageArgs<double>{}); else flag(StageArgs<float>{});
  } else if (r.kind == LaunchRec::COL) {
    if (r.f64) flag(ColPtrs<double>{}); else flag(ColPtrs<float>{});
  } else {
    throw HipError(NKREG_EHIP, "only row stages and column passes can be inactive");
  }
  return c;
}

// Equal-shaped sequences for items whose recordings are pairwise ragged-compatible:
// each time loop runs as many iterations as its longest item, and every item that
// has no iteration s gets inactive copies of the longest item's iteration s.
inline std::vector<Recorder> pad_ragged(const std::vector<Recorder>& recs) {
  std::vector<std::vector<SeqBlock>> cuts(recs.size());
  for (size_t i = 0; i < recs.size(); ++i)
    if (!cut_sequence(recs[i], cuts[i]) || cuts[i].size() != cuts[0].size())
      throw HipError(NKREG_EHIP, "sequences without matching time loops");
  const size_t nb = cuts[0].size();
  std::vector<Recorder> out(recs.size());
  for (size_t b = 0; b < nb; ++b) {
    if (cuts[0][b].loop == 0) {
      for (size_t i = 0; i < recs.size(); ++i) {
        const auto rg = cuts[i][b].ranges[0];
        out[i].recs.insert(out[i].recs.end(), recs[i].recs.begin() + rg.first, recs[i].recs.begin() + rg.second);
      }
      continue;
    }
    size_t ref = 0;
    for (size_t i = 1; i < recs.size(); ++i)
      if (cuts[i][b].ranges.size() > cuts[ref][b].ranges.size()) ref = i;
    const size_t iters = cuts[ref][b].ranges.size();
    for (size_t i = 0; i < recs.size(); ++i) {
      for (size_t s = 0; s < iters; ++s) {
        out[i].mark(cuts[0][b].loop, (int)s);
        if (s < cuts[i][b].ranges.size()) {
          const auto rg = cuts[i][b].ranges[s];
          out[i].recs.insert(out[i].recs.end(), recs[i].recs.begin() + rg.first, recs[i].recs.begin() + rg.second);
        } else {
          const auto rg = cuts[ref][b].ranges[s];
          for (size_t k = rg.first; k < rg.second; ++k) out[i].recs.push_back(inactive_copy(recs[ref].recs[k]));
        }
      }
      out[i].mark(LOOP_NONE, 0);
    }
  }
  return out;
}

// The recorded launches of one group of items and where their tables live.
struct GroupPlan {
  std::vector<size_t> items;
  std::vector<Recorder> recs;  // one per item, equal-shaped
  std::vector<size_t> offs;        // per launch position: table offset
  bool ragged = false;             // items with different step counts (padded sequences)
  size_t small_ops = 0;            // leading launches run by the persistent kernel (0: none)
  size_t prog_off = 0;             // table offset of its program
};

// Appends the group's argument tables (items' entries side by side per position).
inline void add_tables(GroupPlan& gp, std::vector<unsigned char>& host) {
  const auto& seq = gp.recs[0].recs;
  gp.offs.assign(seq.size(), 0);
  for (size_t p = 0; p < seq.size(); ++p) {
    if (seq[p].kind == LaunchRec::COPY) continue;
    host.resize((host.size() + 255) / 256 * 256);
    gp.offs[p] = host.size();
    for (const auto& r : gp.recs) host.insert(host.end(), r.recs[p].entry.begin(), r.recs[p].entry.end());
  }
  if (gp.small_ops) {
    const std::vector<SmallOp> prog = small_program(seq, gp.offs, gp.small_ops);
    host.resize((host.size() + 255) / 256 * 256);
    gp.prog_off = host.size();
    const unsigned char* b = reinterpret_cast<const unsigned char*>(prog.data());
    host.insert(host.end(), b, b + prog.size() * sizeof(SmallOp));
  }
}

// Issues the group's launches on st (tables at base).
inline void issue_group(const GroupPlan& gp, void* base, hipStream_t st) {
  const auto& seq = gp.recs[0].recs;
  size_t p0 = 0;
  if (gp.small_ops) {
    const LaunchRec& r0 = first_row(seq);
    unsigned char* b = static_cast<unsigned char*>(base);
    if (!launch_small(r0.f64, small_n1(seq), r0.len, r0.nc1, (int)gp.recs.size(),
                      reinterpret_cast<const SmallOp*>(b + gp.prog_off), (int)gp.small_ops, b, r0.tw, r0.iarg, st))
      throw HipError(-4, "no persistent kernel instance for this grid");
    p0 = gp.small_ops;
  }
  for (size_t p = p0; p < seq.size(); ++p) {
    if (seq[p].kind == LaunchRec::COPY) {
      for (const auto& r : gp.recs) {
        const auto& c = r.recs[p];
        NK_HIP(hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToDevice, st));
      }
    } else {
      launch_group(seq[p], (int)gp.recs.size(), (unsigned char*)base + gp.offs[p], st);
    }
  }
}

// Captures issue_group into a graph on st (which must not be capturing).
inline hipGraphExec_t capture_group(const GroupPlan& gp, void* base, hipStream_t st) {
  hipGraph_t graph = nullptr;
  NK_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  try {
    issue_group(gp, base, st);
  } catch (...) {
    (void)hipStreamEndCapture(st, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  NK_HIP(hipStreamEndCapture(st, &graph));
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) throw HipError(NKREG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  return ex;
}

// Milliseconds per replay of an instantiated graph on st (one warm-up, then two timed).
inline float time_exec(hipGraphExec_t ex, hipStream_t st) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = 0.f;
  try {
    NK_HIP(hipEventCreate(&e0));
    NK_HIP(hipEventCreate(&e1));
    NK_HIP(hipGraphLaunch(ex, st));
    NK_HIP(hipEventRecord(e0, st));
    NK_HIP(hipGraphLaunch(ex, st));
    NK_HIP(hipGraphLaunch(ex, st));
    NK_HIP(hipEventRecord(e1, st));
    NK_HIP(hipEventSynchronize(e1));
    NK_HIP(hipEventElapsedTime(&ms, e0, e1));
  } catch (...) {
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / 2.f;
}

// Milliseconds per replay of the group's launches (one warm-up, then two timed).
inline float time_group(const GroupPlan& gp, hipStream_t st) {
  std::vector<unsigned char> host;
  GroupPlan g = gp;
  add_tables(g, host);
  void* dev = nullptr;
  if (!host.empty()) {
    NK_HIP(hipMalloc(&dev, host.size()));
    NK_HIP(hipMemcpy(dev, host.data(), host.size(), hipMemcpyHostToDevice));
  }
  hipGraphExec_t ex = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = 0.f;
  try {
    ex = capture_group(g, dev, st);
    NK_HIP(hipEventCreate(&e0));
    NK_HIP(hipEventCreate(&e1));
    NK_HIP(hipGraphLaunch(ex, st));
    NK_HIP(hipEventRecord(e0, st));
    NK_HIP(hipGraphLaunch(ex, st));
    NK_HIP(hipGraphLaunch(ex, st));
    NK_HIP(hipEventRecord(e1, st));
    NK_HIP(hipEventSynchronize(e1));
    NK_HIP(hipEventElapsedTime(&ms, e0, e1));
  } catch (...) {
    (void)hipStreamSynchronize(st);
    if (ex) (void)hipGraphExecDestroy(ex);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (dev) (void)hipFree(dev);
    throw;
  }
  (void)hipGraphExecDestroy(ex);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (dev) (void)hipFree(dev);
  return ms / 2.f;
}


// The faster of a set of candidate plans for one group (every candidate gives the same
// values): each is replayed at the group's scale and timed; ms[i] receives the times.
inline size_t fastest_plan(const std::vector<GroupPlan>& cands, hipStream_t st, std::vector<float>* ms = nullptr) {
  size_t best = 0;
  float tbest = 0.f;
  if (ms) ms->clear();
  if (small_forced()) {
    if (ms) ms->assign(cands.size(), 0.f);
    for (size_t i = 0; i < cands.size(); ++i)
      if (cands[i].small_ops) return i;
  }
  for (size_t i = 0; i < cands.size(); ++i) {
    const float t = time_group(cands[i], st);
    if (ms) ms->push_back(t);
    if (i == 0 || t < tbest) {
      tbest = t;
      best = i;
    }
  }
  return best;
}

}  // namespace nk
