// Batched launches: many independent (kind, n, P) products.  One launch
// covers the work items of one pass whose transforms have the same size, for
// every instance of that size (hmv_batch_launches counts them: 24 for the
// 256-instance mix of four precisions).  hmv_batch_matvec_single runs the
// whole batch as one cooperative launch with grid-wide barriers between the
// passes.  Also the host-side sizing, descriptors and item lists.  A single
// persistent launch with a device work queue and dependency counters is kept
// in the source but switched off: it did not finish on two runs and the
// cause is unknown.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "common.h"
#include "hmv.h"
#include "kernels.h"
#include "plan.h"
#include "tables.h"

using namespace hmv;

namespace {

constexpr int kBatchMaxN = 2048;       // index axis <= 4096 points: both halves fit in LDS
int g_spin_limit = 1000000;            // dependency waits are bounded (about a second)
// The single persistent launch (work queue + per-instance counters) is
// switched off; batches run as one launch per pass.
constexpr bool kBatchPersistent = false;

struct InstPlan {
  FftSizes z;
  int64_t off_h1, off_hh, off_x1, off_y1;
};

// Limb width of a batch instance from the worst-case bound (no data read):
// every digit of h and x at magnitude 2^(w-1).
// With allow3 the row passes take limb transforms of 3 * 2^k points where
// those are smaller; the single-launch forms have power-of-two rows only.
bool batch_inst_sizes(int64_t n, int32_t P, bool allow3, FftSizes* out) {
  if (n < 1 || n > kBatchMaxN) return false;
  for (int w = kFftWMax; w >= kFftWMin; --w) {
    FftSizes z;
    if (!fft_sizes(n, P, w, &z, allow3)) continue;
    const double nh = std::ldexp(1.0, w - 1) * std::sqrt((double)(2 * n - 1) * (double)z.L);
    const double nx = std::ldexp(1.0, w - 1) * std::sqrt((double)n * (double)z.L);
    // stages as for a plan without the shared column (fft_bound_for)
    const int k = z.z3 ? z.logNt + z.logM + 2 + 1 + 2 : z.logNt + (z.logM + 1) + 2;
    const double b = fft_conv_bound(nh, nx, k, fft_twiddle_beta());
    const double cmax = (double)n * z.L * std::ldexp(1.0, 2 * (w - 1));
    const int NC = 2 * z.L - 1;
    const size_t carry_end = (size_t)(NC * 8 + 15) / 16 * 16 + (size_t)carry_lds_bytes(kBatchThreads);
    if (b < 0.5 && cmax < std::ldexp(1.0, 50) && carry_end <= kBatchDynLds) {
      *out = z;
      return true;
    }
  }
  return false;
}

struct BatchLayout {
  int64_t off_ctr, off_inst, off_items, off_data, total;
  int nitems;
  std::vector<InstPlan> ip;
};

bool batch_layout(const hmv_problem* probs, int32_t count, bool allow3, BatchLayout* L) {
  if (!probs || count < 1) return false;
  L->ip.resize(count);
  int64_t items = 0;
  for (int i = 0; i < count; ++i) {
    const hmv_problem& pr = probs[i];
    if (!valid_kind(pr.kind) || pr.P < 1 || pr.P > HMV_MAX_P) return false;
    if (!batch_inst_sizes(pr.n, pr.P, allow3, &L->ip[i].z)) return false;
    items += 3 * pr.n - 1 + 2 * L->ip[i].z.C + pr.n;
  }
  if (items > INT32_MAX / 2) return false;
  L->nitems = (int)items;
  int64_t off = kStatusBytes;
  L->off_ctr = off;
  off = align_up(off + 4 * (1 + 4 * (int64_t)count));
  L->off_inst = off;
  off = align_up(off + (int64_t)sizeof(BatchInst) * count);
  L->off_items = off;
  off = align_up(off + 16 * items);
  L->off_data = off;
  for (int i = 0; i < count; ++i) {
    const int64_t n = probs[i].n;
    const FftSizes& z = L->ip[i].z;
    const int64_t tile_elems = 8 * (int64_t)z.tiles;
    L->ip[i].off_h1 = off;
    off = align_up(off + 16 * tile_elems * (2 * n - 1));
    L->ip[i].off_hh = off;
    off = align_up(off + 16 * (int64_t)z.C * z.Nt);
    L->ip[i].off_x1 = off;
    off = align_up(off + 16 * tile_elems * n);
    L->ip[i].off_y1 = off;
    off = align_up(off + 16 * tile_elems * n);
  }
  L->total = off;
  return true;
}

// Status clear, instance descriptors and the pass-major item list, uploaded
// into the workspace.  Within a pass the items are grouped by transform size
// (largest first) and, inside a size, by instance cost.  runs gets one entry
// per (pass, size); starts[p] is the first item of pass p.
struct Run { int phase, logn, start, count; };

int batch_prepare(const hmv_problem* probs, int32_t count, const BatchLayout& L, char* base,
                  hipStream_t s, std::vector<Run>* runs, int starts[4]) {
  DevStatus* st = reinterpret_cast<DevStatus*>(base);
  hipError_t e = launch_clear_status(st, s);
  if (e != hipSuccess) return status_from_hip(e, "clear status");
  std::vector<BatchInst> inst(count);
  for (int i = 0; i < count; ++i) {
    const hmv_problem& pr = probs[i];
    const FftSizes& z = L.ip[i].z;
    BatchInst& b = inst[i];
    b.h = pr.h;
    b.x = pr.x;
    b.y = pr.y;
    b.H1 = reinterpret_cast<double2*>(base + L.ip[i].off_h1);
    b.Hh = reinterpret_cast<double2*>(base + L.ip[i].off_hh);
    b.X1 = reinterpret_cast<double2*>(base + L.ip[i].off_x1);
    b.Y1 = reinterpret_cast<double2*>(base + L.ip[i].off_y1);
    b.n = (int)pr.n;
    b.P = pr.P;
    b.W = (int)words_of(pr.P);
    b.w = z.w;
    b.L = z.L;
    b.logM = z.logM;
    b.logNt = z.logNt;
    b.C = z.C;
    b.gather = pr.kind == HMV_CIRCULANT ? (int)pr.n : 0;
    b.reverse = pr.kind == HMV_HANKEL ? 0 : (int)pr.n;   // reversal block: the n rows
    b.scale = z.z3 ? std::ldexp(1.0 / 3.0, -(z.logNt + z.logM))
                   : std::ldexp(1.0, -(z.logNt + z.logM + 1));
  }
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::vector<int4> items;
  items.reserve(L.nitems);
  for (int ph = 0; ph < 4; ++ph) {
    starts[ph] = (int)items.size();
    auto logn_of = [&](int i) {
      const FftSizes& z = L.ip[i].z;
      return (ph == 0 || ph == 3) ? z.logM + (z.z3 ? kBatchLog3 : 0) : z.logNt - 1;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      if (logn_of(a) != logn_of(b)) return logn_of(a) > logn_of(b);
      return (int64_t)probs[a].n * L.ip[a].z.C > (int64_t)probs[b].n * L.ip[b].z.C;
    });
    for (int i : order) {
      const int logn = logn_of(i);
      if (runs->empty() || runs->back().phase != ph || runs->back().logn != logn)
        runs->push_back({ph, logn, (int)items.size(), 0});
      const int cnt = ph == 0 ? 3 * (int)probs[i].n - 1
                      : ph == 3 ? (int)probs[i].n
                                : L.ip[i].z.C;
      for (int r = 0; r < cnt; ++r) items.push_back(make_int4(i, ph, r, 0));
      runs->back().count += cnt;
    }
  }
  e = hipMemcpyAsync(base + L.off_inst, inst.data(), sizeof(BatchInst) * count,
                     hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + L.off_items, items.data(), 16 * items.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);     // host lists must outlive the copies
  if (e != hipSuccess) return status_from_hip(e, "batch upload");
  return HMV_OK;
}

int batch_check(const hmv_problem* probs, int32_t count, bool allow3, void* ws, int64_t ws_bytes,
                BatchLayout* L) {
  if (!batch_layout(probs, count, allow3, L)) return HMV_EINVAL;
  for (int i = 0; i < count; ++i)
    if (!probs[i].h || !probs[i].x || !probs[i].y) return HMV_EINVAL;
  if (!ws || ws_bytes < L->total) return HMV_ENOMEM;
  return HMV_OK;
}

}  // namespace

extern "C" {

int64_t hmv_batch_workspace_bytes(const hmv_problem* probs, int32_t count) {
  BatchLayout L;
  if (!batch_layout(probs, count, !kBatchPersistent, &L)) return HMV_EINVAL;
  return L.total;
}

int64_t hmv_batch_single_workspace_bytes(const hmv_problem* probs, int32_t count) {
  BatchLayout L;
  if (!batch_layout(probs, count, false, &L)) return HMV_EINVAL;
  return L.total;
}

int hmv_batch_matvec(const hmv_problem* probs, int32_t count, void* ws, int64_t ws_bytes,
                     void* stream) {
  const bool allow3 = !kBatchPersistent;
  BatchLayout L;
  int rc = batch_check(probs, count, allow3, ws, ws_bytes, &L);
  if (rc != HMV_OK) return rc;
  clear_stale_error();
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  std::vector<Run> runs;
  int starts[4];
  rc = batch_prepare(probs, count, L, base, s, &runs, starts);
  if (rc != HMV_OK) return rc;
  DevStatus* st = reinterpret_cast<DevStatus*>(base);
  const BatchInst* d_inst = reinterpret_cast<const BatchInst*>(base + L.off_inst);
  const int4* d_items = reinterpret_cast<const int4*>(base + L.off_items);
  hipError_t e = hipSuccess;
  if (kBatchPersistent) {
    int dev = 0, cus = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return status_from_hip(e, "device query");
    const int grid = std::max(1, std::min(2 * cus, L.nitems));
    int* head = reinterpret_cast<int*>(base + L.off_ctr);
    e = launch_batch(d_inst, d_items, L.nitems, head, head + 1, 4 * count, grid, g_spin_limit, st, s);
    return status_from_hip(e, "batch kernel");
  }
  // one launch per pass and transform size
  for (const Run& r : runs) {
    if (e != hipSuccess) break;
    e = launch_batch_phase(r.phase, r.logn, d_inst, d_items + r.start, r.count, st, s);
  }
  return status_from_hip(e, "batch kernels");
}

int hmv_batch_matvec_single(const hmv_problem* probs, int32_t count, void* ws, int64_t ws_bytes,
                            void* stream) {
  BatchLayout L;
  int rc = batch_check(probs, count, false, ws, ws_bytes, &L);
  if (rc != HMV_OK) return rc;
  clear_stale_error();
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  std::vector<Run> runs;
  int starts[4];
  rc = batch_prepare(probs, count, L, base, s, &runs, starts);
  if (rc != HMV_OK) return rc;
  hipError_t e = launch_batch_coop(reinterpret_cast<const BatchInst*>(base + L.off_inst),
                                   reinterpret_cast<const int4*>(base + L.off_items), starts,
                                   L.nitems, reinterpret_cast<DevStatus*>(base), nullptr, s);
  return status_from_hip(e, "batch cooperative kernel");
}

int32_t hmv_batch_launches(const hmv_problem* probs, int32_t count) {
  BatchLayout L;
  if (!batch_layout(probs, count, !kBatchPersistent, &L)) return HMV_EINVAL;
  std::vector<int> limb, index;
  for (int i = 0; i < count; ++i) {
    limb.push_back(L.ip[i].z.logM + (L.ip[i].z.z3 ? kBatchLog3 : 0));
    index.push_back(L.ip[i].z.logNt - 1);
  }
  std::sort(limb.begin(), limb.end());
  std::sort(index.begin(), index.end());
  const int nl = (int)(std::unique(limb.begin(), limb.end()) - limb.begin());
  const int ni = (int)(std::unique(index.begin(), index.end()) - index.begin());
  return 2 * nl + 2 * ni;
}

int hmv_debug_batch_spin_limit(int32_t spins) {
  if (spins < 0) return HMV_EINVAL;
  g_spin_limit = spins > 0 ? spins : 1000000;
  return HMV_OK;
}

}  // extern "C"
