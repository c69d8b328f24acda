// Many independent problems in one time loop: grouped, persistent stage launches per
// kernel class, captured once per step into a HIP graph; launch shapes chosen by
// timing candidates on the problems' own data.
//
// Classes.  Constant-coefficient problems group by (arithmetic type, N+1): they share
// one specialisation of the fused stage kernel (fdm.hip), whose tiles of EPB elements
// are spread over a persistent grid.  PCG problems group by N+1 and share one block
// size of the PCG stage kernel (pcg.hip), one element per block iteration.
//
// Tuning.  For every class the candidates (EPB and grid size for the constant path,
// block size and grid size for PCG) are timed on stage 1 of the class's own problems.
// Stage 1 writes only the stage register Y and the second trace buffer, which the next
// real step overwrites first, so the problems' states are untouched; the PCG warm starts
// and iteration counters of the timing runs go to scratch copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"

using namespace gdw;

namespace {

struct FdmClass {
  int elem_bytes = 8;
  int n1 = 0;
  int epb = 1;
  unsigned grid = 0;
  std::vector<int> members;
  void* d_args[4] = {nullptr, nullptr, nullptr, nullptr};
  long* d_tiles = nullptr;
};

struct PcgClass {
  int n1 = 0;
  int threads = 1024;
  size_t lds = 0;
  unsigned grid = 0;
  std::vector<int> members;
  PcgStageArgs* d_args[4] = {nullptr, nullptr, nullptr, nullptr};
  long* d_el = nullptr;
  // split stage (register-operator families): d_args[k] holds the members' arguments
  // followed by those of the mapped members again (the M_J solves walk only these)
  bool split = false;
  int n_mapped = 0;
  long* d_el_m = nullptr;
  std::vector<long> h_el, h_el_m;   // host copies of d_el, d_el_m
};

}  // namespace

struct gdw_batch {
  std::vector<gdw_ctx*> ctx;
  std::vector<FdmClass> fdm;
  std::vector<PcgClass> pcg;
  std::vector<double> dt;      // per-problem dt of the instantiated graph
  long long epoch = -1;        // sum of the members' argument epochs at graph build
  hipStream_t cap = nullptr;   // private stream used for graph capture
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipEvent_t> ev;  // step boundaries of the last run
  int last_steps = 0;
  int tuned = 0;
  int ncu = 256;
  std::string plan;
};

static void drop_graph(gdw_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

static void free_classes(gdw_batch* b) {
  for (auto& c : b->fdm) {
    for (auto& p : c.d_args) if (p) (void)hipFree(p);
    if (c.d_tiles) (void)hipFree(c.d_tiles);
  }
  for (auto& c : b->pcg) {
    for (auto& p : c.d_args) if (p) (void)hipFree(p);
    if (c.d_el) (void)hipFree(c.d_el);
    if (c.d_el_m) (void)hipFree(c.d_el_m);
  }
}

// ---------------------------------------------------------------------------------
// argument tables
// ---------------------------------------------------------------------------------
template <typename T>
static gdw_status upload_fdm_args(gdw_batch* b, FdmClass& c, int stage,
                                  const std::vector<double>& dt) {
  std::vector<StageArgs<T>> h;
  for (int i : c.members) h.push_back(fdm_stage_args<T>(b->ctx[i], stage, dt[i]));
  void*& d = c.d_args[stage - 1];
  if (!d) GDW_HIP(hipMalloc(&d, h.size() * sizeof(StageArgs<T>)));
  GDW_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(StageArgs<T>), hipMemcpyHostToDevice));
  return GDW_OK;
}

static gdw_status upload_fdm_tiles(FdmClass& c, const std::vector<gdw_ctx*>& ctx) {
  std::vector<long> t(c.members.size() + 1, 0);
  for (size_t k = 0; k < c.members.size(); ++k)
    t[k + 1] = t[k] + (ctx[c.members[k]]->nel + c.epb - 1) / c.epb;
  if (!c.d_tiles) GDW_HIP(hipMalloc(&c.d_tiles, t.size() * sizeof(long)));
  GDW_HIP(hipMemcpy(c.d_tiles, t.data(), t.size() * sizeof(long), hipMemcpyHostToDevice));
  return GDW_OK;
}

static long fdm_tiles(const FdmClass& c, const std::vector<gdw_ctx*>& ctx, int epb) {
  long t = 0;
  for (int i : c.members) t += (ctx[i]->nel + epb - 1) / epb;
  return t;
}

static long pcg_elems(const PcgClass& c, const std::vector<gdw_ctx*>& ctx) {
  long t = 0;
  for (int i : c.members) t += ctx[i]->nel;
  return t;
}

// PCG stage arguments for a block size; `scratch` (if non-empty) redirects the warm
// starts and counters of member k to scratch[k] (xS, xM, its, fail).
struct PcgScratch { double* xS; double* xM; int* its; int* fail; };

static gdw_status upload_pcg_args(gdw_batch* b, PcgClass& c, int stage,
                                  const std::vector<double>& dt, int threads,
                                  const std::vector<PcgScratch>* scratch, size_t* lds_out) {
  std::vector<PcgStageArgs> h;
  size_t lds = 0;
  for (size_t k = 0; k < c.members.size(); ++k) {
    const gdw_ctx* x = b->ctx[c.members[k]];
    PcgStageArgs a = pcg_stage_args(x, stage, dt[c.members[k]]);
    size_t l;
    if (!pcg_args_shape(a, threads, &l)) l = (size_t)-1;   // block too small: not a candidate
    lds = std::max(lds, l);
    if (scratch) {
      a.xS = (*scratch)[k].xS;
      a.xM = (*scratch)[k].xM;
      a.its = (*scratch)[k].its;
      a.fail = (*scratch)[k].fail;
    }
    h.push_back(a);
  }
  PcgStageArgs*& d = c.d_args[stage - 1];
  if (!d) GDW_HIP(hipMalloc(&d, h.size() * sizeof(PcgStageArgs)));
  GDW_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(PcgStageArgs), hipMemcpyHostToDevice));
  *lds_out = lds;
  return GDW_OK;
}

// Mapped members of a split class, in member order.
static std::vector<int> mapped_members(const PcgClass& c, const std::vector<gdw_ctx*>& ctx) {
  std::vector<int> m;
  for (int i : c.members)
    if (ctx[i]->d.mapped) m.push_back(i);
  return m;
}

static gdw_status upload_split_args(gdw_batch* b, PcgClass& c, int stage,
                                    const std::vector<double>& dt) {
  std::vector<PcgStageArgs> h;
  for (int i : c.members) h.push_back(pcg_stage_args(b->ctx[i], stage, dt[i]));
  for (int i : mapped_members(c, b->ctx)) h.push_back(pcg_stage_args(b->ctx[i], stage, dt[i]));
  PcgStageArgs*& d = c.d_args[stage - 1];
  if (!d) GDW_HIP(hipMalloc(&d, h.size() * sizeof(PcgStageArgs)));
  GDW_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(PcgStageArgs), hipMemcpyHostToDevice));
  return GDW_OK;
}

static gdw_status upload_split_el(PcgClass& c, const std::vector<gdw_ctx*>& ctx) {
  const std::vector<int> m = mapped_members(c, ctx);
  std::vector<long> t(m.size() + 1, 0);
  for (size_t k = 0; k < m.size(); ++k) t[k + 1] = t[k] + ctx[m[k]]->nel;
  c.n_mapped = (int)m.size();
  c.h_el_m = t;
  c.h_el.assign(c.members.size() + 1, 0);
  for (size_t k = 0; k < c.members.size(); ++k) c.h_el[k + 1] = c.h_el[k] + ctx[c.members[k]]->nel;
  if (!c.d_el_m) GDW_HIP(hipMalloc(&c.d_el_m, t.size() * sizeof(long)));
  GDW_HIP(hipMemcpy(c.d_el_m, t.data(), t.size() * sizeof(long), hipMemcpyHostToDevice));
  return GDW_OK;
}

// A register-operator class runs the split stage when every member has its lift buffers and
// the members share the block layout (a function of N, p and the precision, so equal
// layouts mean equal unit tables).
static bool split_class(const PcgClass& c, const std::vector<gdw_ctx*>& ctx) {
  if (!pcg_split_key(c.n1) || c.members.empty()) return false;
  const gdw_ctx* x0 = ctx[c.members[0]];
  for (int i : c.members) {
    const gdw_ctx* x = ctx[i];
    if (!x->Fu || !x->Fv || x->n1 != x0->n1 || x->d.p != x0->d.p ||
        x->blk_threads != x0->blk_threads || x->blk_K != x0->blk_K || x->blk_CH != x0->blk_CH ||
        x->blk_WB != x0->blk_WB)
      return false;
  }
  return true;
}

static hipError_t launch_split_class(gdw_batch* b, const PcgClass& c, int stage,
                                     const std::vector<double>& dt, hipStream_t st) {
  const PcgStageArgs h = pcg_stage_args(b->ctx[c.members[0]], stage, dt[c.members[0]]);
  const int np = (int)c.members.size();
  const PcgStageArgs* d = c.d_args[stage - 1];
  return launch_pcg_split_group(stage, c.n1, d, c.d_el, c.h_el.data(), np, d + np, c.d_el_m,
                                c.h_el_m.data(), c.n_mapped, h, c.threads, st);
}

static gdw_status upload_pcg_el(PcgClass& c, const std::vector<gdw_ctx*>& ctx) {
  std::vector<long> t(c.members.size() + 1, 0);
  for (size_t k = 0; k < c.members.size(); ++k) t[k + 1] = t[k] + ctx[c.members[k]]->nel;
  if (!c.d_el) GDW_HIP(hipMalloc(&c.d_el, t.size() * sizeof(long)));
  GDW_HIP(hipMemcpy(c.d_el, t.data(), t.size() * sizeof(long), hipMemcpyHostToDevice));
  return GDW_OK;
}

static hipError_t launch_fdm_class(const FdmClass& c, int stage, int epb, unsigned grid,
                                   hipStream_t st) {
  const int np = (int)c.members.size();
  if (c.elem_bytes == 8)
    return launch_stage_group<double>(stage, c.n1, epb, (const StageArgs<double>*)c.d_args[stage - 1],
                                      c.d_tiles, np, grid, st);
  return launch_stage_group<float>(stage, c.n1, epb, (const StageArgs<float>*)c.d_args[stage - 1],
                                   c.d_tiles, np, grid, st);
}

// ---------------------------------------------------------------------------------
// tuning
// ---------------------------------------------------------------------------------
// Mean time (ms) of `reps` launches after one warm-up.
template <typename F>
static gdw_status time_launch(F&& f, hipStream_t st, int reps, float* ms) {
  hipEvent_t e0, e1;
  GDW_HIP(hipEventCreate(&e0));
  GDW_HIP(hipEventCreate(&e1));
  hipError_t e = f();
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = f();
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) {
    set_error(std::string("batch tuning: ") + hipGetErrorString(e));
    return GDW_EHIP;
  }
  *ms = t / reps;
  return GDW_OK;
}

// Launch shapes chosen by the tuner, kept for the life of the process and keyed by the
// device architecture, the path, the arithmetic type, the kernel family and the sizes of the
// class's members: a later batch with a class of the same key takes the shape untimed.
struct TunedShape {
  int a = 0;            // FDM: elements per tile; PCG: block size
  unsigned grid = 0;
  size_t lds = 0;
};

static std::mutex g_tune_mu;
static std::map<std::string, TunedShape> g_tuned;

static std::string tune_key(const char* path, int elem_bytes, int family,
                            const std::vector<int>& members, const std::vector<gdw_ctx*>& ctx) {
  int dev = 0;
  hipDeviceProp_t prop{};
  std::string k = "?";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    k = prop.gcnArchName;
  k += std::string("|") + path + "|" + std::to_string(elem_bytes) + "|" + std::to_string(family);
  for (int i : members) k += "|" + std::to_string(ctx[i]->nel);
  return k;
}

static bool tuned_lookup(const std::string& key, TunedShape* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tuned.find(key);
  if (it == g_tuned.end()) return false;
  *out = it->second;
  return true;
}

static void tuned_store(const std::string& key, const TunedShape& v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = v;
}

static gdw_status tune_fdm(gdw_batch* b, FdmClass& c, const std::vector<double>& dt,
                           hipStream_t st, std::string& log) {
  char buf[160];
  const std::string key = tune_key("fdm", c.elem_bytes, c.n1, c.members, b->ctx);
  TunedShape ts;
  if (tuned_lookup(key, &ts)) {
    (void)dt;
    (void)st;
    c.epb = ts.a;
    c.grid = ts.grid;
    std::snprintf(buf, sizeof buf, "  fdm n1=%d %s: epb=%d grid=%u (cached)\n", c.n1,
                  c.elem_bytes == 8 ? "f64" : "f32", c.epb, c.grid);
    log += buf;
    return upload_fdm_tiles(c, b->ctx);
  }
  float best = 1e30f;
  int best_epb = 0;
  unsigned best_grid = 0;
  for (int epb : {1, 2, 4, 8}) {
    if (stage_lds_bytes(c.n1, epb) > 65536) continue;
    c.epb = epb;
    gdw_status s;
    if ((s = upload_fdm_tiles(c, b->ctx)) != GDW_OK) return s;
    if (c.elem_bytes == 8) s = upload_fdm_args<double>(b, c, 1, dt);
    else s = upload_fdm_args<float>(b, c, 1, dt);
    if (s != GDW_OK) return s;
    const long tiles = fdm_tiles(c, b->ctx, epb);
    const int occ = c.elem_bytes == 8 ? stage_group_occupancy<double>(1, c.n1, epb)
                                      : stage_group_occupancy<float>(1, c.n1, epb);
    std::vector<unsigned> grids = {(unsigned)std::min<long>(tiles, (long)occ * b->ncu),
                                   (unsigned)std::min<long>(tiles, 2L * occ * b->ncu),
                                   (unsigned)tiles};
    std::sort(grids.begin(), grids.end());
    grids.erase(std::unique(grids.begin(), grids.end()), grids.end());
    for (unsigned grid : grids) {
      float ms;
      s = time_launch([&]() { return launch_fdm_class(c, 1, epb, grid, st); }, st, 3, &ms);
      if (s != GDW_OK) return s;
      std::snprintf(buf, sizeof buf, "  fdm n1=%d %s epb=%d grid=%u: %.4f ms\n", c.n1,
                    c.elem_bytes == 8 ? "f64" : "f32", epb, grid, ms);
      log += buf;
      if (ms < best) { best = ms; best_epb = epb; best_grid = grid; }
    }
  }
  if (!best_epb) { set_error("no launch shape fits this class"); return GDW_EUNSUPPORTED; }
  c.epb = best_epb;
  c.grid = best_grid;
  ts.a = best_epb;
  ts.grid = best_grid;
  tuned_store(key, ts);
  return upload_fdm_tiles(c, b->ctx);
}

static gdw_status tune_pcg(gdw_batch* b, PcgClass& c, const std::vector<double>& dt,
                           hipStream_t st, std::string& log) {
  if (c.split) {
    // persistent grids sized by occupancy; the block layout fixes the block sizes
    (void)dt;
    (void)st;
    gdw_status s;
    if ((s = upload_pcg_el(c, b->ctx)) != GDW_OK || (s = upload_split_el(c, b->ctx)) != GDW_OK)
      return s;
    c.threads = b->ctx[c.members[0]]->blk_threads;
    c.grid = 0;
    c.lds = 0;
    char buf[160];
    std::snprintf(buf, sizeof buf, "  pcg key=%d: split stage, %d of %zu members mapped\n", c.n1,
                  c.n_mapped, c.members.size());
    log += buf;
    return GDW_OK;
  }
  const std::string key = tune_key("pcg", 8, c.n1, c.members, b->ctx);
  TunedShape ts;
  if (tuned_lookup(key, &ts)) {
    gdw_status s2;
    if ((s2 = upload_pcg_el(c, b->ctx)) != GDW_OK) return s2;
    c.threads = ts.a;
    c.grid = ts.grid;
    c.lds = ts.lds;
    char buf2[160];
    std::snprintf(buf2, sizeof buf2, "  pcg key=%d: threads=%d grid=%u lds=%zu (cached)\n", c.n1,
                  c.threads, c.grid, c.lds);
    log += buf2;
    return GDW_OK;
  }
  // scratch warm starts / counters (copies of the real ones)
  std::vector<PcgScratch> scr;
  gdw_status s = GDW_OK;
  for (int i : c.members) {
    const gdw_ctx* x = b->ctx[i];
    const size_t nodal = (size_t)x->nel * x->g.nn * sizeof(double);
    PcgScratch p{};
    if (hipMalloc(&p.xS, nodal) != hipSuccess || hipMalloc(&p.xM, nodal) != hipSuccess ||
        hipMalloc(&p.its, (size_t)x->nel * kItsPer * sizeof(int)) != hipSuccess ||
        hipMalloc(&p.fail, sizeof(int)) != hipSuccess) {
      scr.push_back(p);
      s = GDW_ENOMEM;
      set_error("batch tuning: scratch allocation failed");
      break;
    }
    scr.push_back(p);
    (void)hipMemcpyAsync(p.xS, x->xS, nodal, hipMemcpyDeviceToDevice, st);
    (void)hipMemcpyAsync(p.xM, x->xM, nodal, hipMemcpyDeviceToDevice, st);
    (void)hipMemsetAsync(p.its, 0, (size_t)x->nel * kItsPer * sizeof(int), st);
    (void)hipMemsetAsync(p.fail, 0x7f, sizeof(int), st);
  }
  float best = 1e30f;
  int best_thr = 0;
  unsigned best_grid = 0;
  size_t best_lds = 0;
  char buf[160];
  int nn_max = 0;
  for (int i : c.members)
    nn_max = std::max(nn_max, std::max(b->ctx[i]->g.nn, b->ctx[i]->blk_threads));
  const long els = pcg_elems(c, b->ctx);
  if (s == GDW_OK && (s = upload_pcg_el(c, b->ctx)) == GDW_OK) {
    for (int thr : {1024, 768, 512, 256}) {
      if (thr < ((nn_max + 63) / 64) * 64 || thr > pcg_group_max_threads(c.n1)) continue;
      size_t lds;
      if ((s = upload_pcg_args(b, c, 1, dt, thr, &scr, &lds)) != GDW_OK) break;
      if (lds > 160 * 1024) continue;
      const int occ = std::max(1, std::min((int)((160 * 1024) / lds), 2048 / thr));
      std::vector<unsigned> grids = {(unsigned)std::min<long>(els, (long)occ * b->ncu),
                                     (unsigned)els};
      std::sort(grids.begin(), grids.end());
      grids.erase(std::unique(grids.begin(), grids.end()), grids.end());
      for (unsigned grid : grids) {
        float ms;
        s = time_launch([&]() {
              return launch_pcg_stage_group(1, c.n1, c.d_args[0], c.d_el, (int)c.members.size(),
                                            grid, thr, lds, st);
            }, st, 1, &ms);
        if (s != GDW_OK) break;
        std::snprintf(buf, sizeof buf, "  pcg key=%d threads=%d grid=%u lds=%zu: %.4f ms\n",
                      c.n1, thr, grid, lds, ms);
        log += buf;
        if (ms < best) { best = ms; best_thr = thr; best_grid = grid; best_lds = lds; }
      }
      if (s != GDW_OK) break;
    }
  }
  (void)hipStreamSynchronize(st);
  for (auto& p : scr) {
    if (p.xS) (void)hipFree(p.xS);
    if (p.xM) (void)hipFree(p.xM);
    if (p.its) (void)hipFree(p.its);
    if (p.fail) (void)hipFree(p.fail);
  }
  if (s != GDW_OK) return s;
  if (!best_thr) { set_error("no launch shape fits this PCG class"); return GDW_EUNSUPPORTED; }
  c.threads = best_thr;
  c.grid = best_grid;
  c.lds = best_lds;
  ts.a = best_thr;
  ts.grid = best_grid;
  ts.lds = best_lds;
  tuned_store(key, ts);
  return GDW_OK;
}

static gdw_status build_graph(gdw_batch* b, const std::vector<double>& dt) {
  drop_graph(b);
  gdw_status s;
  for (auto& c : b->fdm)
    for (int k = 1; k <= 4; ++k) {
      s = c.elem_bytes == 8 ? upload_fdm_args<double>(b, c, k, dt) : upload_fdm_args<float>(b, c, k, dt);
      if (s != GDW_OK) return s;
    }
  for (auto& c : b->pcg)
    for (int k = 1; k <= 4; ++k) {
      if (c.split) {
        if ((s = upload_split_args(b, c, k, dt)) != GDW_OK) return s;
        continue;
      }
      size_t lds;
      if ((s = upload_pcg_args(b, c, k, dt, c.threads, nullptr, &lds)) != GDW_OK) return s;
      c.lds = std::max(c.lds, lds);
    }
  GDW_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  // source terms: each member's step weights from its device clock, before the stages
  for (size_t i = 0; i < b->ctx.size() && e == hipSuccess; ++i) {
    gdw_ctx* x = b->ctx[i];
    if (x->nf > 0) e = launch_source_step(x->t_dev, x->t_dev + 1, dt[i], source_terms(x), b->cap);
  }
  for (int k = 1; k <= 4 && e == hipSuccess; ++k) {
    for (auto& c : b->fdm) {
      if ((e = launch_fdm_class(c, k, c.epb, c.grid, b->cap)) != hipSuccess) break;
    }
    for (auto& c : b->pcg) {
      if (e != hipSuccess) break;
      if (c.split) e = launch_split_class(b, c, k, dt, b->cap);
      else e = launch_pcg_stage_group(k, c.n1, c.d_args[k - 1], c.d_el, (int)c.members.size(),
                                      c.grid, c.threads, c.lds, b->cap);
    }
  }
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    set_error(std::string("batch graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    return GDW_EHIP;
  }
  b->graph = g;
  GDW_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  b->dt = dt;
  b->epoch = 0;
  for (const gdw_ctx* c : b->ctx) b->epoch += c->args_epoch;
  return GDW_OK;
}

static void make_plan(gdw_batch* b, const std::string& log) {
  std::string p;
  char buf[200];
  for (auto& c : b->fdm) {
    std::snprintf(buf, sizeof buf, "fdm n1=%d %s: %zu problems, epb=%d grid=%u\n", c.n1,
                  c.elem_bytes == 8 ? "f64" : "f32", c.members.size(), c.epb, c.grid);
    p += buf;
  }
  for (auto& c : b->pcg) {
    char fam[48];
    if (c.n1 == 0) std::snprintf(fam, sizeof fam, "rows");
    else if (c.n1 & 64)
      std::snprintf(fam, sizeof fam, "blocks n1=%d (registers, p=%d%s)", c.n1 & 31, c.n1 >> 7,
                    b->ctx[c.members[0]]->d.precision == GDW_MIXED_PC32 ? ", FP32 chain" : "");
    else if (c.n1 & 32) std::snprintf(fam, sizeof fam, "mixed n1=%d", c.n1 & 31);
    else std::snprintf(fam, sizeof fam, "blocks n1=%d", c.n1 & 31);
    if (c.split)
      std::snprintf(buf, sizeof buf, "pcg %s: %zu problems, split stage (%d mapped)\n", fam,
                    c.members.size(), c.n_mapped);
    else
      std::snprintf(buf, sizeof buf, "pcg %s: %zu problems, threads=%d grid=%u lds=%zu\n", fam,
                    c.members.size(), c.threads, c.grid, c.lds);
    p += buf;
  }
  b->plan = p + "candidates:\n" + log;
}

// ---------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------
extern "C" gdw_status gdw_batch_create(int nprob, const gdw_desc* descs, gdw_batch** out) {
  if (!out || !descs) { set_error("NULL argument"); return GDW_EINVAL; }
  *out = nullptr;
  if (nprob <= 0 || nprob > 4096) { set_error("nprob must be in [1, 4096]"); return GDW_EINVAL; }
  gdw_batch* b = new (std::nothrow) gdw_batch();
  if (!b) { set_error("host allocation failed"); return GDW_ENOMEM; }
  gdw_status s = GDW_OK;
  for (int i = 0; i < nprob && s == GDW_OK; ++i) {
    if (descs[i].dim == 3) {
      set_error("problem " + std::to_string(i) + ": 3D problems are not batched");
      s = GDW_EUNSUPPORTED;
      break;
    }
    gdw_ctx* c = nullptr;
    s = gdw_create(&descs[i], &c);
    if (s == GDW_OK) b->ctx.push_back(c);
    else set_error("problem " + std::to_string(i) + ": " + gdw_last_error());
  }
  int dev = 0;
  if (s == GDW_OK && (hipGetDevice(&dev) != hipSuccess ||
                      hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
                          hipSuccess ||
                      hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)) {
    set_error("batch: device query or stream creation failed");
    s = GDW_EHIP;
  }
  if (s == GDW_OK) {
    std::map<std::pair<int, int>, size_t> fk, pk;
    for (int i = 0; i < nprob; ++i) {
      const gdw_ctx* c = b->ctx[i];
      if (c->solver == GDW_SOLVE_PCG) {
        // kernel family (the grouped kernel's key): layout, precision and, for the
        // register-operator kernels, the degree
        const int fam = pcg_family_key(c->n1, c->d.p, c->blk_v2,
                                       c->d.precision == GDW_MIXED_FP32);
        // (the FP32 preconditioner chain is a kernel variant of its family)
        auto key = std::make_pair(fam, c->d.precision == GDW_MIXED_PC32 ? 1 : 0);
        if (!pk.count(key)) { pk[key] = b->pcg.size(); b->pcg.emplace_back(); b->pcg.back().n1 = fam; }
        b->pcg[pk[key]].members.push_back(i);
      } else {
        auto key = std::make_pair((int)c->elem_bytes, c->n1);
        if (!fk.count(key)) {
          fk[key] = b->fdm.size();
          b->fdm.emplace_back();
          b->fdm.back().elem_bytes = (int)c->elem_bytes;
          b->fdm.back().n1 = c->n1;
        }
        b->fdm[fk[key]].members.push_back(i);
      }
    }
  }
  for (auto& c : b->pcg) c.split = split_class(c, b->ctx);
  if (s == GDW_OK && !b->pcg.empty() && pcg_group_prepare() != hipSuccess) {
    set_error("batch: cannot raise the LDS limit of the PCG stage kernels");
    s = GDW_EHIP;
  }
  if (s != GDW_OK) {
    gdw_batch_destroy(b);
    return s;
  }
  *out = b;
  return GDW_OK;
}

extern "C" gdw_status gdw_batch_ctx(gdw_batch* b, int i, gdw_ctx** ctx) {
  if (!b || !ctx) { set_error("NULL argument"); return GDW_EINVAL; }
  if (i < 0 || i >= (int)b->ctx.size()) { set_error("problem index out of range"); return GDW_EINVAL; }
  *ctx = b->ctx[i];
  return GDW_OK;
}

static gdw_status check_ready(gdw_batch* b, const double* dt) {
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    if (!b->ctx[i]->have_state) {
      set_error("problem " + std::to_string(i) + " has no state: call gdw_set_state first");
      return GDW_EINVAL;
    }
    if (!(dt[i] > 0) || !std::isfinite(dt[i])) {
      set_error("problem " + std::to_string(i) + ": dt must be finite and > 0");
      return GDW_EINVAL;
    }
  }
  return GDW_OK;
}

extern "C" gdw_status gdw_batch_tune(gdw_batch* b, const double* dt, void* stream) {
  if (!b || !dt) { set_error("NULL argument"); return GDW_EINVAL; }
  gdw_status s = check_ready(b, dt);
  if (s != GDW_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> d(dt, dt + b->ctx.size());
  std::string log;
  for (auto& c : b->fdm)
    if ((s = tune_fdm(b, c, d, st, log)) != GDW_OK) return s;
  for (auto& c : b->pcg)
    if ((s = tune_pcg(b, c, d, st, log)) != GDW_OK) return s;
  GDW_HIP(hipStreamSynchronize(st));
  make_plan(b, log);
  b->tuned = 1;
  drop_graph(b);
  return GDW_OK;
}

extern "C" gdw_status gdw_batch_run(gdw_batch* b, const double* dt, int steps, void* stream) {
  if (!b || !dt) { set_error("NULL argument"); return GDW_EINVAL; }
  if (steps < 0) { set_error("steps must be >= 0"); return GDW_EINVAL; }
  gdw_status s = check_ready(b, dt);
  if (s != GDW_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (!b->tuned && (s = gdw_batch_tune(b, dt, stream)) != GDW_OK) return s;
  std::vector<double> d(dt, dt + b->ctx.size());
  long long ep = 0;
  for (const gdw_ctx* c : b->ctx) ep += c->args_epoch;
  if (!b->exec || d != b->dt || ep != b->epoch) {
    GDW_HIP(hipStreamSynchronize(st));
    if ((s = build_graph(b, d)) != GDW_OK) return s;
  }
  for (auto e : b->ev) (void)hipEventDestroy(e);
  b->ev.assign(steps + 1, nullptr);
  for (auto& e : b->ev) GDW_HIP(hipEventCreate(&e));
  for (int k = 0; k < steps; ++k) {
    GDW_HIP(hipEventRecord(b->ev[k], st));
    GDW_HIP(hipGraphLaunch(b->exec, st));
  }
  GDW_HIP(hipEventRecord(b->ev[steps], st));
  b->last_steps = steps;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    gdw_ctx* c = b->ctx[i];
    c->steps_taken += steps;
    c->t += steps * d[i];   // host mirror of the source clock (the device clock advanced)
    if (c->solver == GDW_SOLVE_PCG) c->stages_since_state += 4LL * steps;
  }
  return GDW_OK;
}

extern "C" gdw_status gdw_batch_step_times(gdw_batch* b, float* ms, int n) {
  if (!b || (!ms && n > 0)) { set_error("NULL argument"); return GDW_EINVAL; }
  if (n != b->last_steps) { set_error("n must equal the step count of the last gdw_batch_run"); return GDW_EINVAL; }
  if (n == 0) return GDW_OK;
  GDW_HIP(hipEventSynchronize(b->ev[n]));
  for (int k = 0; k < n; ++k) GDW_HIP(hipEventElapsedTime(&ms[k], b->ev[k], b->ev[k + 1]));
  return GDW_OK;
}

extern "C" const char* gdw_batch_plan(gdw_batch* b) { return b ? b->plan.c_str() : ""; }

extern "C" void gdw_batch_destroy(gdw_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  drop_graph(b);
  for (auto e : b->ev) (void)hipEventDestroy(e);
  free_classes(b);
  for (gdw_ctx* c : b->ctx) gdw_destroy(c);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}
