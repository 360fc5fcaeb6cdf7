// lbfz_batch.hip -- the batched sweep of the C ABI (include/lbfz.h): many
// independent 2D grids, each a complete solver state (its own parameters,
// size, buffers and totals), advanced together.
//
// One step of the batch is one launch of k_step2d_batch over a single work
// table of (grid, tile) items that spans every grid, whatever its size, with
// the grids' kernel parameters and per-parity buffers in a device table: the
// tiles of the small grids, too few to fill the GPU on their own, run beside
// those of the large ones.  The tile height (4 or 8 rows) and the launch
// shape (one block per item, or a persistent grid of 2, 4 or 8 blocks per CU
// looping over the items) are chosen by a timing search of the whole step
// (lbfz_batch_tune).  Steps are replayed from a HIP graph captured once per
// configuration: a graph of graph_steps steps holds one kernel node per step.
// Grids of equal size form a group (reported by lbfz_batch_group_config).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/lbfz.h"
#include "lbfz_common.hpp"
#include "lbfz_handle.hpp"
#include "lbfz_kernels.hpp"

using namespace lbfz;

namespace {

constexpr int kGraphSteps = 12;  // steps per captured graph (a multiple of 2 and 3)
constexpr int kTY[2] = {4, 8};

struct Group {
  int nx, ny;
  std::vector<int> cases;
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int slots_of(int storage) { return storage == LBFZ_STORE_F32 ? 2 : 6; }

}  // namespace

struct lbfz_batch {
  int ncases = 0;
  int storage = 0;
  int L = 2;  // parity slots of the step arguments
  std::vector<lbfz_handle*> h;
  std::vector<Group> groups;
  hipStream_t stream = nullptr;  // caller's
  hipStream_t cap = nullptr;     // capture stream (internal)
  BatchCase* d_cases = nullptr;
  std::vector<BatchCase> cases;  // host copy of the table
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int64_t step = 0;
  EquilJob* d_jobs = nullptr;  // device table of a batched restart (ncases entries)
  std::vector<char> selected;  // per grid: advanced by the steps
  std::vector<char> stale;     // per grid: left behind by a subset step
  int nwork[2] = {0, 0};       // work items of every grid at tile height kTY[v]
  int2* work[2] = {nullptr, nullptr};  // device work tables (every grid)
  int nsel[2] = {0, 0};        // the same for the selected grids
  int2* sel[2] = {nullptr, nullptr};
  bool all = true;             // every grid selected: launch over work[], else sel[]
  int ty_index = 0;            // chosen tile height (index into kTY)
  int grid = 0;                // blocks per launch; 0: one per work item
};

namespace {

#define HIPCHK(x)                            \
  do {                                       \
    if ((x) != hipSuccess) return LBFZ_EHIP; \
  } while (0)

// Case table entry of grid i for tile height ty: the handle's parameters with
// that tiling, and the step arguments of every parity slot.
void fill_case(lbfz_batch* b, int i, int ty) {
  lbfz_handle* h = b->h[i];
  BatchCase& c = b->cases[i];
  c.P = h->kp;
  int nbx, nby;
  c.P.nblk = tiles2d(h->kp.nx, h->kp.ny, &nbx, &nby, ty);
  c.P.nblk_x = nbx;
  c.P.nblk_y = nby;
  const int cur = h->cur;
  const int64_t step = h->step;
  for (int k = 0; k < b->L; ++k) {
    h->step = k;
    h->cur = k & 1;
    c.A[k] = base_args(h);
  }
  h->step = step;
  h->cur = cur;
}

int upload_cases(lbfz_batch* b) {
  for (int i = 0; i < b->ncases; ++i) fill_case(b, i, kTY[b->ty_index]);
  HIPCHK(hipMemcpyAsync(b->d_cases, b->cases.data(), sizeof(BatchCase) * b->ncases,
                        hipMemcpyHostToDevice, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  return LBFZ_OK;
}

// One step of every selected grid: one launch over the work table.
hipError_t launch_all(lbfz_batch* b, int64_t step, hipStream_t st) {
  const int v = b->ty_index;
  const int n = b->all ? b->nwork[v] : b->nsel[v];
  if (n == 0) return hipSuccess;  // no grid selected
  return launch_step2d_batch(b->storage, kTY[v], b->d_cases, b->all ? b->work[v] : b->sel[v], n,
                             b->grid, (int)(step % b->L), st);
}

// XCD-aware order of a flat (grid, tile) item list: item e runs on the XCD
// e % 8, which gets a contiguous band of the flat list.
std::vector<int2> xcd_order(const std::vector<int2>& flat) {
  const int n = (int)flat.size();
  std::vector<int2> tab(n);
  const int band = n >> 3;
  for (int e = 0; e < n; ++e)
    tab[e] = (band == 0 || (n & 7)) ? flat[e] : flat[(e & 7) * band + (e >> 3)];
  return tab;
}

// Items of every grid for which keep(grid) holds, tile height kTY[v]: the
// grids group by group, each grid's tiles contiguous, then XCD-ordered.
template <class F>
std::vector<int2> batch_items(const lbfz_batch* b, int v, F keep) {
  std::vector<int2> flat;
  for (const Group& g : b->groups) {
    int nbx, nby;
    const int per = tiles2d(g.nx, g.ny, &nbx, &nby, kTY[v]);
    for (int c : g.cases)
      if (keep(c))
        for (int t = 0; t < per; ++t) flat.push_back(make_int2(c, t));
  }
  return xcd_order(flat);
}

void drop_graph(lbfz_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Capture kGraphSteps steps (starting at a step that is 0 mod L) of every
// grid on the capture stream: one kernel node per step.
int build_graph(lbfz_batch* b) {
  drop_graph(b);
  HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (int s = 0; s < kGraphSteps && e == hipSuccess; ++s) e = launch_all(b, s, b->cap);
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->cap, &graph);
  if (e != hipSuccess || e2 != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    return LBFZ_EHIP;
  }
  b->graph = graph;
  if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
    drop_graph(b);
    return LBFZ_EHIP;
  }
  return LBFZ_OK;
}

// A step over the selection: every selected grid must be current; the grids
// left out fall behind the batch's time level.
int begin_step(lbfz_batch* b, int64_t nsteps) {
  for (int i = 0; i < b->ncases; ++i)
    if (b->selected[i] && b->stale[i]) return LBFZ_EINVAL;
  if (nsteps > 0)
    for (int i = 0; i < b->ncases; ++i)
      if (!b->selected[i]) b->stale[i] = 1;
  return LBFZ_OK;
}

void sync_handles(lbfz_batch* b) {
  for (lbfz_handle* h : b->h) {
    h->step = b->step;
    h->cur = (int)(b->step & 1);
  }
}

}  // namespace

extern "C" {

int lbfz_batch_workspace_bytes(int32_t ncases, const lbfz_params* params, size_t* bytes) {
  if (ncases <= 0 || !params || !bytes) return LBFZ_EINVAL;
  size_t total = 0, items = 0;
  for (int i = 0; i < ncases; ++i) {
    if (params[i].dim != 2 || params[i].storage != params[0].storage) return LBFZ_EINVAL;
    size_t w = 0;
    const int rc = lbfz_workspace_bytes(&params[i], &w);
    if (rc != LBFZ_OK) return rc;
    total += align256(w);
    int nbx, nby;
    for (int ty : kTY) items += (size_t)tiles2d(params[i].nx, params[i].ny, &nbx, &nby, ty);
  }
  total += align256(sizeof(BatchCase) * (size_t)ncases);
  // work and selection tables of every grid, for each tile height
  total += 2 * align256(sizeof(int2) * items) + 4 * 256;
  total += align256(sizeof(EquilJob) * (size_t)ncases);
  *bytes = total;
  return LBFZ_OK;
}

int lbfz_batch_create(int32_t ncases, const lbfz_params* params, const double* const* phi,
                      const double* const* T, const double* const* C, void* d_workspace,
                      size_t ws_bytes, void* stream, lbfz_batch** out) {
  if (!out) return LBFZ_EINVAL;
  *out = nullptr;
  size_t need = 0;
  const int rc0 = lbfz_batch_workspace_bytes(ncases, params, &need);
  if (rc0 != LBFZ_OK) return rc0;
  if (!phi || !T || !C || !d_workspace) return LBFZ_EINVAL;
  if (ws_bytes < need || ((uintptr_t)d_workspace & 255)) return LBFZ_ENOMEM;
  lbfz_batch* b = new (std::nothrow) lbfz_batch;
  if (!b) return LBFZ_ENOMEM;
  b->ncases = ncases;
  b->storage = params[0].storage;
  b->L = slots_of(b->storage);
  b->stream = (hipStream_t)stream;
  char* q = (char*)d_workspace;
  int rc = LBFZ_OK;
  for (int i = 0; i < ncases && rc == LBFZ_OK; ++i) {
    size_t w = 0;
    lbfz_workspace_bytes(&params[i], &w);
    lbfz_handle* h = nullptr;
    rc = lbfz_create(&params[i], phi[i], T[i], C[i], nullptr, q, w, stream, &h);
    if (rc == LBFZ_OK) b->h.push_back(h);
    q += align256(w);
  }
  if (rc != LBFZ_OK) {
    lbfz_batch_destroy(b);
    return rc;
  }
  b->d_cases = (BatchCase*)q;
  q += align256(sizeof(BatchCase) * (size_t)ncases);
  b->cases.resize(ncases);
  b->selected.assign(ncases, 1);
  b->stale.assign(ncases, 0);
  // groups of equal grid size, in order of first appearance
  std::map<std::pair<int, int>, int> gid;
  for (int i = 0; i < ncases; ++i) {
    const auto key = std::make_pair(params[i].nx, params[i].ny);
    auto it = gid.find(key);
    if (it == gid.end()) {
      it = gid.emplace(key, (int)b->groups.size()).first;
      Group g;
      g.nx = params[i].nx;
      g.ny = params[i].ny;
      b->groups.push_back(g);
    }
    b->groups[it->second].cases.push_back(i);
  }
  // work tables: (grid, tile) items of every grid in an XCD-aware order (item
  // e runs on the XCD e % 8, which gets a contiguous band of the item list)
  for (int v = 0; v < 2; ++v) {
    const std::vector<int2> tab = batch_items(b, v, [](int) { return true; });
    const int n = (int)tab.size();
    b->nwork[v] = n;
    b->work[v] = (int2*)q;
    q += align256(sizeof(int2) * (size_t)n);
    b->nsel[v] = 0;
    b->sel[v] = (int2*)q;  // room for a selection of every grid
    q += align256(sizeof(int2) * (size_t)n);
    if (hipMemcpyAsync(b->work[v], tab.data(), sizeof(int2) * n, hipMemcpyHostToDevice,
                       b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
      lbfz_batch_destroy(b);
      return LBFZ_EHIP;
    }
  }
  b->d_jobs = (EquilJob*)q;
  q += align256(sizeof(EquilJob) * (size_t)ncases);
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    b->cap = nullptr;
    lbfz_batch_destroy(b);
    return LBFZ_EHIP;
  }
  rc = upload_cases(b);
  if (rc != LBFZ_OK) {
    lbfz_batch_destroy(b);
    return rc;
  }
  *out = b;
  return LBFZ_OK;
}

int lbfz_batch_tune(lbfz_batch* b, int32_t trial_steps) {
  if (!b || trial_steps <= 0) return LBFZ_EINVAL;
  {
    const int rc = begin_step(b, trial_steps);
    if (rc != LBFZ_OK) return rc;
  }
  // candidates: tile height (waves per block) x launch shape (one block per
  // item, or a persistent grid of blocks_per_cu blocks on each CU)
  struct Cand {
    int v, per_cu;
  };
  const Cand cands[] = {{0, 0}, {1, 0}, {0, 2}, {0, 4}, {0, 8}, {1, 2}, {1, 4}, {1, 8}};
  const int nc = (int)(sizeof(cands) / sizeof(cands[0]));
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (cus <= 0) cus = 256;
  float best = 1e30f;
  Cand pick = cands[0];
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // every candidate runs trial_steps real steps of every selected grid; the
  // results do not depend on the candidate (the per-node arithmetic is the
  // same)
  for (int k = 0; k < nc; ++k) {
    b->ty_index = cands[k].v;
    b->grid = cands[k].per_cu * cus;
    int rc = upload_cases(b);
    if (rc != LBFZ_OK) return rc;
    HIPCHK(hipEventRecord(e0, b->stream));
    for (int s = 0; s < trial_steps; ++s) HIPCHK(launch_all(b, b->step + s, b->stream));
    HIPCHK(hipEventRecord(e1, b->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      pick = cands[k];
    }
    b->step += trial_steps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->ty_index = pick.v;
  b->grid = pick.per_cu * cus;
  drop_graph(b);
  sync_handles(b);
  return upload_cases(b);
}

int lbfz_batch_step(lbfz_batch* b, int64_t nsteps) {
  if (!b || nsteps < 0) return LBFZ_EINVAL;
  {
    const int rc = begin_step(b, nsteps);
    if (rc != LBFZ_OK) return rc;
  }
  auto one = [&]() -> int {
    HIPCHK(launch_all(b, b->step, b->stream));
    b->step += 1;
    return LBFZ_OK;
  };
  while (nsteps > 0 && b->step % kGraphSteps != 0) {
    const int rc = one();
    if (rc != LBFZ_OK) return rc;
    --nsteps;
  }
  // graphs for the full selection only: a subset (the screening's fallback)
  // changes every stride, and its launches are cheaper than a capture
  bool all = true;
  for (char c : b->selected) all = all && c;
  if (all && nsteps >= kGraphSteps) {
    if (!b->exec) {
      const int rc = build_graph(b);
      if (rc != LBFZ_OK) return rc;
    }
    while (nsteps >= kGraphSteps) {
      HIPCHK(hipGraphLaunch(b->exec, b->stream));
      b->step += kGraphSteps;
      nsteps -= kGraphSteps;
    }
  }
  while (nsteps > 0) {
    const int rc = one();
    if (rc != LBFZ_OK) return rc;
    --nsteps;
  }
  sync_handles(b);
  return LBFZ_OK;
}

int lbfz_batch_step_sequential(lbfz_batch* b, int64_t nsteps) {
  if (!b || nsteps < 0) return LBFZ_EINVAL;
  {
    const int rc = begin_step(b, nsteps);
    if (rc != LBFZ_OK) return rc;
  }
  sync_handles(b);
  for (int i = 0; i < b->ncases; ++i) {
    if (!b->selected[i]) continue;
    const int rc = lbfz_step(b->h[i], nsteps);
    if (rc != LBFZ_OK) return rc;
  }
  b->step += nsteps;
  sync_handles(b);
  return LBFZ_OK;
}

int lbfz_batch_groups(lbfz_batch* b) { return b ? (int)b->groups.size() : LBFZ_EINVAL; }

int lbfz_batch_group_config(lbfz_batch* b, int32_t group, int32_t* nx, int32_t* ny,
                            int32_t* ncases, int32_t* tile_rows, int32_t* grid_blocks) {
  if (!b || group < 0 || group >= (int)b->groups.size()) return LBFZ_EINVAL;
  const Group& g = b->groups[group];
  if (nx) *nx = g.nx;
  if (ny) *ny = g.ny;
  if (ncases) *ncases = (int32_t)g.cases.size();
  if (tile_rows) *tile_rows = kTY[b->ty_index];
  if (grid_blocks) *grid_blocks = b->grid;
  return LBFZ_OK;
}

int lbfz_batch_fields(lbfz_batch* b, int32_t i, uint32_t field_mask, float* const* dst,
                      int dst_is_device) {
  if (!b || i < 0 || i >= b->ncases || b->stale[i]) return LBFZ_EINVAL;
  sync_handles(b);
  return lbfz_fields(b->h[i], field_mask, dst, dst_is_device);
}

int lbfz_batch_fields_all(lbfz_batch* b, uint32_t field_mask, float* d_dst, int64_t case_stride) {
  if (!b || !d_dst || field_mask == 0 || (field_mask >> 9) != 0) return LBFZ_EINVAL;
  int nf = 0;
  for (int k = 0; k < 9; ++k) nf += (field_mask >> k) & 1;
  for (int i = 0; i < b->ncases; ++i) {
    const int64_t N = (int64_t)b->h[i]->kp.N;
    if (b->stale[i] || case_stride < nf * N) return LBFZ_EINVAL;
  }
  sync_handles(b);
  // one dry-pass launch over every (grid, tile) item
  const int slot = (int)(b->step % b->L);
  const int v = b->ty_index;
  HIPCHK(launch_fields2d_batch(b->storage, kTY[v], b->d_cases, b->work[v], b->nwork[v], slot,
                               d_dst, (long)case_stride, field_mask, b->stream));
  return LBFZ_OK;
}

int lbfz_batch_totals(lbfz_batch* b, int32_t i, lbfz_totals_t* out) {
  if (!b || i < 0 || i >= b->ncases || b->stale[i]) return LBFZ_EINVAL;
  sync_handles(b);
  return lbfz_totals(b->h[i], out);
}

int lbfz_batch_select(lbfz_batch* b, int32_t n, const int32_t* idx) {
  if (!b || n < 0 || (n > 0 && !idx)) return LBFZ_EINVAL;
  std::vector<char> sel(b->ncases, n == 0 ? 1 : 0);
  for (int k = 0; k < n; ++k) {
    if (idx[k] < 0 || idx[k] >= b->ncases) return LBFZ_EINVAL;
    sel[idx[k]] = 1;
  }
  b->selected = sel;
  b->all = true;
  for (char c : sel) b->all = b->all && c;
  if (!b->all) {
    for (int v = 0; v < 2; ++v) {
      const std::vector<int2> tab = batch_items(b, v, [&](int c) { return sel[c] != 0; });
      b->nsel[v] = (int)tab.size();
      if (b->nsel[v] > 0)
        HIPCHK(hipMemcpyAsync(b->sel[v], tab.data(), sizeof(int2) * tab.size(),
                              hipMemcpyHostToDevice, b->stream));
    }
  }
  HIPCHK(hipStreamSynchronize(b->stream));
  // the captured graph (all grids, full work tables) stays valid: subsets
  // are stepped with plain launches
  return LBFZ_OK;
}

int lbfz_batch_restart_many(lbfz_batch* b, int32_t n, const int32_t* idx,
                            const float* const* d_fields, const int64_t* case_stride) {
  if (!b || n < 0 || (n > 0 && (!idx || !d_fields || !case_stride))) return LBFZ_EINVAL;
  // the device job table holds ncases entries: at most one job per grid
  if (n > b->ncases) return LBFZ_EINVAL;
  {
    std::vector<char> seen(b->ncases, 0);
    for (int k = 0; k < n; ++k) {
      if (idx[k] < 0 || idx[k] >= b->ncases || seen[idx[k]]) return LBFZ_EINVAL;
      seen[idx[k]] = 1;
    }
  }
  sync_handles(b);
  if (n == 0) return LBFZ_OK;
  if (b->storage == LBFZ_STORE_F32) {
    // FP32 storage: every grid's restart in one launch (a job table)
    std::vector<EquilJob> jobs(n);
    long max_n = 0;
    for (int k = 0; k < n; ++k) {
      const float* f[7];
      for (int m = 0; m < 7; ++m) f[m] = d_fields[m] + idx[k] * case_stride[m];
      const int rc = restart_job(b->h[idx[k]], f, &jobs[k]);
      if (rc != LBFZ_OK) return rc;
      max_n = std::max<long>(max_n, jobs[k].P.N);
    }
    HIPCHK(hipMemcpyAsync(b->d_jobs, jobs.data(), sizeof(EquilJob) * n, hipMemcpyHostToDevice,
                          b->stream));
    for (int k0 = 0; k0 < n; k0 += 65535)
      HIPCHK(launch_equil2d_batch(b->d_jobs + k0, std::min(n - k0, 65535), max_n, b->stream));
    // the job table is host memory of this call
    HIPCHK(hipStreamSynchronize(b->stream));
  } else {
    // 16-bit storage: the restart's encoding pass is per grid
    for (int k = 0; k < n; ++k) {
      const float* f[7];
      for (int m = 0; m < 7; ++m) f[m] = d_fields[m] + idx[k] * case_stride[m];
      const int rc = lbfz_restart_fields(b->h[idx[k]], f);
      if (rc != LBFZ_OK) return rc;
    }
  }
  for (int k = 0; k < n; ++k) b->stale[idx[k]] = 0;
  return LBFZ_OK;
}

int lbfz_batch_restart_fields(lbfz_batch* b, int32_t i, const float* const* d_fields) {
  if (!b || i < 0 || i >= b->ncases) return LBFZ_EINVAL;
  sync_handles(b);
  const int rc = lbfz_restart_fields(b->h[i], d_fields);
  if (rc == LBFZ_OK) b->stale[i] = 0;
  return rc;
}

void lbfz_batch_destroy(lbfz_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (lbfz_handle* h : b->h) lbfz_destroy(h);
  delete b;
}

}  // extern "C"
