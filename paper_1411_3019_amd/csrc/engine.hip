// engine.hip -- host engine and C ABI (include/md.h) of the RATTLE + Langevin
// hot path on MI355X.
//
// An Engine holds the device state of one or more jobs (systems) in
// concatenated per-slot arrays, a job table, and the tile lists that let one
// launch cover every resident job.  md_ctx is an Engine with one job; md_pool
// is an Engine with many.
//
// Time stepping: chunks of k step launches are captured once into a hipGraph
// and replayed; the device flags a job whose neighbour list would go stale
// (accumulated maximum displacement above skin/2) and skips its remaining
// launches; after each chunk the host reads the per-job bookkeeping, rebuilds
// the lists of the jobs that need it and chooses the next chunk length from
// the observed displacement rate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/md.h"
#include "kernels.hpp"
#include "launch.hpp"

using namespace mdk;

namespace {

constexpr int kDefaultKmax = 16;   // list capacity (a multiple of kRow)
constexpr int kDefaultHcap = 640;  // halo capacity per tile
constexpr int kMaxHcap = 16128;    // window entries are 14-bit (bead-model entries carry a type)
constexpr int kMaxChunk = 64;
constexpr int kPoolChunk = 32;
constexpr size_t kArenaBytes = (size_t)4 << 20;  // pinned staging for small uploads

#define HIPCHK(expr)                   \
  do {                                 \
    hipError_t e_ = (expr);            \
    if (e_ != hipSuccess) {            \
      (void)hipGetLastError();         \
      return MD_EHIP;                  \
    }                                  \
  } while (0)

#define MDCHK(expr)        \
  do {                     \
    int r_ = (expr);       \
    if (r_ != MD_OK) return r_; \
  } while (0)

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// First-fit allocator over an index range (particle slots, bitmap words).
// ---------------------------------------------------------------------------
class FirstFit {
 public:
  void reset(int64_t cap) {
    free_.clear();
    if (cap > 0) free_[0] = cap;
    cap_ = cap;
  }
  int64_t alloc(int64_t len, int64_t align) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      const int64_t start = round_up(it->first, align);
      const int64_t end = it->first + it->second;
      if (start + len <= end) {
        const int64_t f0 = it->first;
        free_.erase(it);
        if (start > f0) free_[f0] = start - f0;
        if (start + len < end) free_[start + len] = end - (start + len);
        return start;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t len) {
    if (len <= 0) return;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {
      len += next->second;
      free_.erase(next);
    }
    auto it = free_.lower_bound(off);
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    free_[off] = len;
  }
  int64_t cap() const { return cap_; }

 private:
  std::map<int64_t, int64_t> free_;
  int64_t cap_ = 0;
};

// ---------------------------------------------------------------------------
// Host-side surface evaluation (input validation only).
// ---------------------------------------------------------------------------
int surf_nprm(int kind) {
  switch (kind) {
    case MD_SURF_NONE: return 0;
    case MD_SURF_PLANE: return 6;
    case MD_SURF_SPHERE: return 4;
    case MD_SURF_ELLIPSOID: return 6;
    case MD_SURF_TORUS: return 5;
    case MD_SURF_CYLINDER: return 7;
    case MD_SURF_HEIGHT: return 4;
    case MD_SURF_BRIDGE: return 6;
    default: return -1;
  }
}

// Parameter checks of a surface (shared by single systems and pool jobs).
int validate_surface(int kind, const double* prm, const md_params& p) {
  const int need = surf_nprm(kind);
  if (need < 0 || (need > 0 && !prm)) return MD_EINVAL;
  for (int k = 0; k < need; ++k)
    if (!std::isfinite(prm[k])) return MD_EINVAL;
  if (kind == MD_SURF_SPHERE && !(prm[3] > 0)) return MD_EINVAL;
  if (kind == MD_SURF_ELLIPSOID && !(prm[3] > 0 && prm[4] > 0 && prm[5] > 0)) return MD_EINVAL;
  if (kind == MD_SURF_TORUS && !(prm[3] > prm[4] && prm[4] > 0)) return MD_EINVAL;
  if (kind == MD_SURF_HEIGHT && (!(prm[2] > 0 && prm[3] > 0) || !p.periodic[0] || !p.periodic[1])) return MD_EINVAL;
  if (kind == MD_SURF_BRIDGE) {
    if (!(prm[3] >= 0 && prm[4] > 0 && prm[5] > 0)) return MD_EINVAL;
    for (int k = 1; k < 3; ++k)
      if (p.periodic[k] && p.box_hi[k] - p.box_lo[k] < 2.0 * (prm[4] + prm[5])) return MD_EINVAL;
  }
  return MD_OK;
}

double host_g(int kind, const double* q, const double* x, double* n) {
  const double d0 = x[0] - q[0], d1 = x[1] - q[1], d2 = x[2] - q[2];
  switch (kind) {
    case MD_SURF_PLANE:
      n[0] = q[3], n[1] = q[4], n[2] = q[5];
      return q[3] * d0 + q[4] * d1 + q[5] * d2;
    case MD_SURF_SPHERE:
      n[0] = 2 * d0, n[1] = 2 * d1, n[2] = 2 * d2;
      return d0 * d0 + d1 * d1 + d2 * d2 - q[3] * q[3];
    case MD_SURF_ELLIPSOID: {
      const double a = 1.0 / (q[3] * q[3]), b = 1.0 / (q[4] * q[4]), c = 1.0 / (q[5] * q[5]);
      n[0] = 2 * d0 * a, n[1] = 2 * d1 * b, n[2] = 2 * d2 * c;
      return d0 * d0 * a + d1 * d1 * b + d2 * d2 * c - 1.0;
    }
    case MD_SURF_TORUS: {
      const double rho = std::sqrt(d0 * d0 + d1 * d1);
      const double s = 2.0 * (1.0 - q[3] / rho);
      n[0] = s * d0, n[1] = s * d1, n[2] = 2 * d2;
      return (rho - q[3]) * (rho - q[3]) + d2 * d2 - q[4] * q[4];
    }
    case MD_SURF_CYLINDER:
      n[0] = 2 * q[3] * d0, n[1] = 2 * q[4] * d1, n[2] = 2 * q[5] * d2;
      return q[3] * d0 * d0 + q[4] * d1 * d1 + q[5] * d2 * d2 - q[6] * q[6];
    case MD_SURF_BRIDGE: {
      const double h = 0.5 * q[3], Rb = q[4], R = q[5], c = Rb + R;
      const double r = std::sqrt(d1 * d1 + d2 * d2);
      if (std::fabs(d0) <= h) {
        const double s = R / Rb;
        n[0] = 0, n[1] = -2 * s * d1, n[2] = -2 * s * d2;
        return s * (Rb * Rb - r * r);
      }
      const double sg = d0 > 0 ? 1.0 : -1.0;
      if (r < c) {
        const double f = 2 * (1 - c / r);
        n[0] = 2 * (d0 - sg * h), n[1] = f * d1, n[2] = f * d2;
        return (d0 - sg * h) * (d0 - sg * h) + (r - c) * (r - c) - R * R;
      }
      n[0] = sg * 2 * R, n[1] = 0, n[2] = 0;
      return 2 * R * (std::fabs(d0) - h - R);
    }
    case MD_SURF_HEIGHT: {
      const double kx = 2 * M_PI / q[2], ky = 2 * M_PI / q[3];
      n[0] = -q[1] * kx * std::cos(kx * x[0]) * std::sin(ky * x[1]);
      n[1] = -q[1] * ky * std::sin(kx * x[0]) * std::cos(ky * x[1]);
      n[2] = 1.0;
      return x[2] - q[0] - q[1] * std::sin(kx * x[0]) * std::sin(ky * x[1]);
    }
    default:
      n[0] = n[1] = n[2] = 0;
      return 0;
  }
}

double lj_phi(double eps, double sigma, double r, double* dphi) {
  const double sr = sigma / r;
  const double s6 = sr * sr * sr * sr * sr * sr;
  *dphi = -24.0 * eps * (2.0 * s6 * s6 - s6) / r;
  return 4.0 * eps * (s6 * s6 - s6);
}

int validate_params(const md_params& p) {
  if (!(p.dt > 0.0) || !(p.kT >= 0.0) || !(p.gamma >= 0.0)) return MD_EINVAL;
  if (p.pair_kind < MD_PAIR_NONE || p.pair_kind > MD_PAIR_LJ_SMOOTH) return MD_EINVAL;
  if (p.pair_kind != MD_PAIR_NONE && (!(p.eps >= 0.0) || !(p.sigma > 0.0) || !(p.rc > 0.0))) return MD_EINVAL;
  if (p.skin < 0.0 || p.newton_tol < 0.0 || p.newton_max_iter < 0) return MD_EINVAL;
  if (p.newton_frozen != 0 && p.newton_frozen != 1) return MD_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (p.periodic[k] && !(p.box_hi[k] > p.box_lo[k])) return MD_EINVAL;
  return MD_OK;
}

// Bytes of device state per particle slot (excluding the neighbour list).
constexpr double kInfinityCacheBytes = 256.0 * 1024.0 * 1024.0;  // MI355X last-level (memory-side) cache

constexpr int64_t kSlotBytes = 2 * 24 /*X*/ + 2 * 24 /*P*/ + 2 * 36 /*NZD, NZF*/ + 2 * 4 /*ID*/ + 2 * 1 /*FLG*/ +
                               2 * 8 /*MASS*/ + 24 /*FC*/ + 3 * 24 /*OX,OP,OF*/ + 32 /*OD*/ + 4 /*NCNT*/ +
                               4 * 6 /*rebuild*/ + 16 /*PK*/ + 2 * 1 /*TYPE*/ + 8 /*BW*/;

// Device bytes per slot with list capacity kmax (16-bit entries) and halo
// capacity hcap (per tile of kTile slots).
constexpr double slot_bytes(int kmax, int hcap) {
  return (double)kSlotBytes + 2.0 * kmax + (4.0 * hcap + 4.0) / kTile;
}

struct HostJob {
  bool used = false;
  md_params prm{};
  int surf_kind = MD_SURF_NONE;
  double surf[MD_SURF_MAXPRM] = {0};
  int64_t n = 0, off = 0, seg = 0, bm_off = 0, bm_words = 0;
  JobDev dev{};
  int64_t step = 0, target = 0;
  int64_t last_build = 0, rebuilds = 0;
  bool built = false, done = false, reported = false;
  int status = MD_OK;
  int newton_max = 0, nl_max = 0, halo_max = 0, err_id = -1;
  int64_t err_step = -1;
  int sum_breaches = 0, breach_base = 0;  // breaches so far; those of earlier list epochs
  double nl_sum = 0.0;
  bool lists_pending = false;  // list statistics of the last build not read back yet
  double A_now = 0.0;
  double rate_prev = 0.0;  // displacement per step while the previous list was in use
  double ext_lo[3] = {0, 0, 0}, ext_len[3] = {0, 0, 0};  // region the cell grid covers
  bool have_ext = false;
  double ndof = 0.0;
  bool model = false;  // bead model (record uploaded to DevBufs::models at admission)
  ModelDev mdev{};
};

// Per-job cell grid over the region the particles can occupy.
int make_grid(HostJob& h, const double* x) {
  JobDev& d = h.dev;
  const double rlist = std::sqrt(d.rlist2);
  double lo[3], hi[3];
  bool have[3] = {false, false, false};
  const double* q = h.surf;
  switch (h.surf_kind) {
    case MD_SURF_SPHERE:
      for (int k = 0; k < 3; ++k) lo[k] = q[k] - q[3], hi[k] = q[k] + q[3], have[k] = true;
      break;
    case MD_SURF_ELLIPSOID:
      for (int k = 0; k < 3; ++k) lo[k] = q[k] - q[3 + k], hi[k] = q[k] + q[3 + k], have[k] = true;
      break;
    case MD_SURF_TORUS:
      for (int k = 0; k < 2; ++k) lo[k] = q[k] - q[3] - q[4], hi[k] = q[k] + q[3] + q[4], have[k] = true;
      lo[2] = q[2] - q[4], hi[2] = q[2] + q[4], have[2] = true;
      break;
    case MD_SURF_CYLINDER:
      for (int k = 0; k < 3; ++k)
        if (q[3 + k] != 0.0) lo[k] = q[k] - q[6], hi[k] = q[k] + q[6], have[k] = true;
      break;
    case MD_SURF_HEIGHT:
      lo[2] = q[0] - std::fabs(q[1]), hi[2] = q[0] + std::fabs(q[1]), have[2] = true;
      break;
    default:
      break;
  }
  const bool free_particles = h.surf_kind == MD_SURF_NONE;
  int64_t total = 1;
  for (int k = 0; k < 3; ++k) {
    double a, b;
    if (h.prm.periodic[k]) {
      a = h.prm.box_lo[k];
      b = h.prm.box_hi[k];
      const double L = b - a;
      if (L < 2.0 * rlist) return MD_EINVAL;
      int nc = (int)std::floor(L / rlist);
      nc = std::max(1, std::min(nc, 1 << 20));
      d.nc[k] = nc;
      d.glo[k] = a;
      d.inv_cs[k] = nc / L;
      d.box_len[k] = L;
      d.inv_box_len[k] = 1.0 / L;
      d.periodic[k] = 1;
    } else {
      if (h.prm.box_hi[k] > h.prm.box_lo[k]) {
        a = h.prm.box_lo[k];
        b = h.prm.box_hi[k];
      } else if (have[k] && !free_particles) {
        a = lo[k] - rlist;
        b = hi[k] + rlist;
      } else if (h.have_ext || x == nullptr) {
        // re-planning an existing job (or sizing without particles): keep the region
        a = h.ext_lo[k];
        b = h.ext_lo[k] + h.ext_len[k];
      } else {
        a = b = h.n > 0 ? x[k] : 0.0;
        for (int64_t i = 1; i < h.n; ++i) a = std::min(a, x[3 * i + k]), b = std::max(b, x[3 * i + k]);
        a -= rlist;
        b += rlist;
      }
      const double L = std::max(b - a, rlist);
      int nc = (int)std::floor(L / rlist);
      nc = std::max(1, std::min(nc, 1 << 20));
      d.nc[k] = nc;
      d.glo[k] = a;
      d.inv_cs[k] = nc / L;
      d.box_len[k] = L;
      d.inv_box_len[k] = 1.0 / L;
      d.periodic[k] = 0;
      h.ext_lo[k] = a;
      h.ext_len[k] = L;
    }
    total *= d.nc[k];
  }
  // keep raster indices within 32 bits by coarsening the grid if needed
  while (total > 0xF0000000LL) {
    total = 1;
    for (int k = 0; k < 3; ++k) {
      if (d.nc[k] > 3) {
        const int nc = d.nc[k] / 2;
        d.inv_cs[k] = d.inv_cs[k] * nc / d.nc[k];
        d.nc[k] = nc;
      }
      total *= d.nc[k];
    }
  }
  h.bm_words = total / 32 + 1;  // one spare word: the end of the last z-run is addressable
  h.have_ext = true;
  return MD_OK;
}

struct GraphKey {
  int k;
  bool operator<(const GraphKey& o) const { return k < o.k; }
};

// Scratch of md_get_state_dev_noalloc: the per-block partials of the
// diagnostics reduction (at most kDiagBlocks blocks) and its four results,
// 8224 bytes.  Each device holds its own copy until the process ends; every
// call on a device uses that copy, so such calls must not overlap on one
// device.  Nothing in it needs clearing: each call writes every partial it
// reads.
constexpr int kScratchDoubles = 4 * kDiagBlocks + 4;
static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` per device ordinal (the array's name is a host
// stand-in, not a device address), looked up once per device with that
// device current.
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
double* scratch_dev[kMaxDevices] = {};

int scratch_address(int dev, double** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return MD_EINVAL;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return MD_EHIP;
    }
    scratch_dev[dev] = (double*)ptr;
  }
  *out = scratch_dev[dev];
  return MD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------
struct Engine {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int64_t C = 0;        // slot capacity
  int64_t BMW = 0;      // bitmap word capacity
  int max_jobs = 0;
  int kmax = kDefaultKmax;
  int hcap = kDefaultHcap;
  int lds_max = 65536;  // LDS bytes one workgroup may use on this device
  DevBufs B{};
  std::vector<HostJob> jobs;
  FirstFit slots, words;
  // device scratch for launch descriptors
  // step tile classes, one step kernel each: FP64 forces, FP32 forces, bead
  // model with FP64 forces, bead model with FP32 forces; + 4: the same for jobs
  // on the height field or the bridge (kernels built with every surface)
  static constexpr int kClasses = 8;
  int* step_tiles_job = nullptr;       // [kClasses][tile_cap]
  int64_t* step_tiles_first = nullptr;
  int* step_counts = nullptr;          // [kClasses]: tiles in each list (read by the step kernels)
  int grid[kClasses] = {};             // grid sizes baked into the cached graphs
  int f32_variant = 0;                 // FP32-class step-kernel instance (kStepVariants; md_tune)
  bool stream_stores = false;          // store policy of the step and list kernels (set_store_policy)
  int* aux_tiles_job = nullptr;        // rebuild / finish lists
  int64_t* aux_tiles_first = nullptr;
  int64_t tile_cap = 0;
  Chunk* chunks_d = nullptr;
  uint32_t* chunk_sums = nullptr;
  double* diag_d = nullptr;  // [4 kDiagBlocks] partials, then [4] results
  uint32_t* kkey_d = nullptr;  // list build: window records of FP64-class / bead-model tiles that do not fit LDS
  int64_t kkey_cap = 0;
  bool list_table_global = false;  // MD_LIST_TABLE_GLOBAL: keep those records in global memory always
  bool scan_three_pass = false;    // MD_SCAN_3PASS: the three-pass scans whatever the segment lengths
  double* diag_many = nullptr;  // finish_many: [4 kDiagBlocks] diagnostic partials per job
  int64_t diag_many_cap = 0;
  double* pack_d = nullptr;  // finish_many: the results packed for one copy to the host
  int64_t pack_cap = 0;
  char* fj_d = nullptr;  // finish_many: its two job tables
  int64_t fj_cap = 0;
  double* scratch_d = nullptr;  // this device's `scratch` (md_get_state_dev_noalloc)
  bool no_alloc = false;        // set during md_get_state_dev_noalloc: device and pinned allocations fail
  int64_t chunk_cap = 0;
  Range* ranges_d = nullptr;
  int64_t range_cap = 0;
  // pinned host staging
  JobBook* book_h = nullptr;
  char* stage = nullptr;           // bulk transfers (admission, results); free once the stream is drained
  size_t stage_cap = 0;
  char* arena = nullptr;           // small uploads, bump-allocated; recycled when the stream is drained
  size_t arena_used = 0;
  std::map<void*, std::vector<char>> uploaded;  // last contents of descriptor arrays that rarely change
  bool build_timing_pending = false;
  // step graphs (by number of steps), and the stream whole-chunk graphs are
  // captured on while the library's stream runs
  std::map<GraphKey, hipGraphExec_t> graphs;
  hipStream_t cap_stream = nullptr;
  bool step_tiles_valid = false;
  md_stats stats{};
  static constexpr int kSubEvents = 16;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_sub[kSubEvents] = {};
  hipEvent_t ev_book = nullptr;  // the job records of the chunk in flight are on the host
  // the chunk enqueued by launch_chunk and not yet completed (complete_chunk)
  struct Inflight {
    bool active = false;
    std::vector<int64_t> cap;  // steps each job may take in the chunk
    int kk = 0, nsub = 0;
    int64_t launches = 0;
  } inflight;
  std::vector<int> last_tj[kClasses];
  std::vector<int64_t> last_tf[kClasses];
  size_t nl_bytes = 0;

  ~Engine() { release(); }

  void drop_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }

  void release() {
    if (device >= 0) (void)hipSetDevice(device);
    drop_graphs();
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e), e = nullptr;
    for (auto& e : ev_sub)
      if (e) (void)hipEventDestroy(e), e = nullptr;
    if (ev_book) (void)hipEventDestroy(ev_book), ev_book = nullptr;
    void* ptrs[] = {B.X[0], B.X[1], B.P[0], B.P[1], B.ID[0], B.ID[1], B.FLG[0], B.FLG[1], B.MASS[0], B.MASS[1],
                    B.NZD[0], B.NZD[1], B.NZF[0], B.NZF[1], B.FC, B.OX, B.OP, B.OF, B.OD, B.NL, B.NCNT, B.HALO, B.HCNT, B.BM, B.WOFF,
                    B.CCNT, B.CSTART, B.RASTER, B.CID, B.RANK, B.INV, B.BW, B.PK, B.TYPE[0], B.TYPE[1],
                    (void*)B.models, B.TACC, B.NLSTAT, B.jobs, B.book, step_tiles_job, step_tiles_first,
                    step_counts, aux_tiles_job, aux_tiles_first, chunks_d, chunk_sums, ranges_d, diag_d,
                    diag_many, kkey_d, pack_d, fj_d};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    std::memset(&B, 0, sizeof(B));
    step_tiles_job = nullptr;
    step_counts = nullptr;
    step_tiles_first = aux_tiles_first = nullptr;
    aux_tiles_job = nullptr;
    chunks_d = nullptr;
    chunk_sums = nullptr;
    ranges_d = nullptr;
    diag_d = nullptr;
    diag_many = nullptr;
    diag_many_cap = 0;
    pack_d = nullptr;
    pack_cap = 0;
    fj_d = nullptr;
    fj_cap = 0;
    kkey_d = nullptr;
    kkey_cap = 0;
    if (book_h) (void)hipHostFree(book_h);
    if (stage) (void)hipHostFree(stage);
    if (arena) (void)hipHostFree(arena);
    book_h = nullptr;
    stage = nullptr;
    arena = nullptr;
    stage_cap = 0;
    arena_used = 0;
    uploaded.clear();
    if (own_stream && stream) (void)hipStreamDestroy(stream);
    if (cap_stream) (void)hipStreamDestroy(cap_stream), cap_stream = nullptr;
    stream = nullptr;
    own_stream = false;
  }

  template <class T>
  int dalloc(T** p, size_t count) {
    *p = nullptr;
    if (no_alloc) return MD_ENOMEM;
    if (count == 0) count = 1;
    if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return MD_ENOMEM;
    }
    return MD_OK;
  }

  int init(int dev, void* user_stream, int64_t slot_cap, int64_t word_cap, int njobs) {
    device = dev;
    HIPCHK(hipSetDevice(dev));
    MDCHK(scratch_address(dev, &scratch_d));
    if (user_stream) {
      stream = (hipStream_t)user_stream;
      own_stream = false;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
      own_stream = true;
    }
    HIPCHK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
    C = round_up(std::max<int64_t>(slot_cap, kTile), kTile);
    BMW = std::max<int64_t>(word_cap, 64);
    max_jobs = std::max(1, njobs);
    jobs.assign(max_jobs, HostJob());
    slots.reset(C);
    words.reset(BMW);
    B.C = C;
    B.kmax = kmax;
    B.hcap = hcap;
    if (const char* v = std::getenv("MD_LIST_TABLE_GLOBAL")) list_table_global = std::atoi(v) != 0;
    if (const char* v = std::getenv("MD_SCAN_3PASS")) scan_three_pass = std::atoi(v) != 0;
    // MD_NO_BONDED_WINDOW: bonded partners through the inverse permutation only
    if (const char* v = std::getenv("MD_NO_BONDED_WINDOW")) B.no_bw = std::atoi(v) != 0 ? 1 : 0;
    if (const char* v = std::getenv("MD_STEP_VARIANT")) f32_variant = std::max(0, std::min(kNumStepVariants - 1, std::atoi(v)));
    {
      int v = 0;
      if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
        lds_max = v;
      else
        (void)hipGetLastError();
    }
    for (int q = 0; q < 2; ++q) {
      MDCHK(dalloc(&B.X[q], 3 * C));
      MDCHK(dalloc(&B.P[q], 3 * C));
      MDCHK(dalloc(&B.ID[q], C));
      MDCHK(dalloc(&B.FLG[q], C));
      MDCHK(dalloc(&B.MASS[q], C));
      MDCHK(dalloc(&B.NZD[q], 3 * C));
      MDCHK(dalloc(&B.NZF[q], 3 * C));
    }
    MDCHK(dalloc(&B.FC, 3 * C));
    MDCHK(dalloc(&B.OX, 3 * C));
    MDCHK(dalloc(&B.OP, 3 * C));
    MDCHK(dalloc(&B.OF, 3 * C));
    MDCHK(dalloc(&B.OD, 4 * C));
    nl_bytes = (size_t)kmax * C * 2;
    MDCHK(dalloc(&B.NL, (size_t)kmax * C));
    MDCHK(dalloc(&B.NCNT, C));
    MDCHK(dalloc(&B.HALO, (size_t)(C / kTile + 1) * hcap));
    MDCHK(dalloc(&B.HCNT, C / kTile + 1));
    HIPCHK(hipMemsetAsync(B.HCNT, 0, sizeof(uint32_t) * (C / kTile + 1), stream));
    MDCHK(dalloc(&B.BM, BMW));
    MDCHK(dalloc(&B.WOFF, BMW));
    MDCHK(dalloc(&B.CCNT, C));
    MDCHK(dalloc(&B.CSTART, C));
    MDCHK(dalloc(&B.RASTER, C));
    MDCHK(dalloc(&B.CID, C));
    MDCHK(dalloc(&B.RANK, C));
    MDCHK(dalloc(&B.INV, C));
    MDCHK(dalloc(&B.BW, C));
    MDCHK(dalloc(&B.PK, C + 16));  // the list build reads up to 7 records past a column
    MDCHK(dalloc(&B.TYPE[0], C));
    MDCHK(dalloc(&B.TYPE[1], C));
    MDCHK(dalloc(&B.TACC, C / kGroup + 1));
    HIPCHK(hipMemsetAsync(B.TACC, 0, sizeof(double) * (C / kGroup + 1), stream));
    MDCHK(dalloc(&B.jobs, max_jobs));
    {
      ModelDev* md = nullptr;
      MDCHK(dalloc(&md, max_jobs));
      B.models = md;
    }
    MDCHK(dalloc(&B.book, max_jobs));
    {
      std::vector<JobBook> fresh(max_jobs, fresh_book());
      HIPCHK(hipMemcpy(B.book, fresh.data(), sizeof(JobBook) * max_jobs, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemsetAsync(B.NCNT, 0, sizeof(uint32_t) * C, stream));
    tile_cap = C / kTile + max_jobs + 8;
    MDCHK(dalloc(&B.NLSTAT, 2 * (C / kGroup + 1)));
    HIPCHK(hipMemsetAsync(B.NLSTAT, 0, sizeof(uint32_t) * 2 * (C / kGroup + 1), stream));
    MDCHK(dalloc(&step_tiles_job, kClasses * tile_cap));
    MDCHK(dalloc(&step_tiles_first, kClasses * tile_cap));
    MDCHK(dalloc(&step_counts, kClasses));
    HIPCHK(hipMemsetAsync(step_counts, 0, kClasses * sizeof(int), stream));
    MDCHK(dalloc(&aux_tiles_job, tile_cap));
    MDCHK(dalloc(&aux_tiles_first, tile_cap));
    chunk_cap = (C + max_jobs) / kScanChunk + BMW / kScanChunk + 4 * max_jobs + 16;
    MDCHK(dalloc(&chunks_d, chunk_cap));
    MDCHK(dalloc(&chunk_sums, chunk_cap));
    MDCHK(dalloc(&diag_d, 4 * kDiagBlocks + 4));
    range_cap = 3 * max_jobs + 4;
    MDCHK(dalloc(&ranges_d, range_cap));
    HIPCHK(hipHostMalloc((void**)&book_h, sizeof(JobBook) * max_jobs, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&arena, kArenaBytes, hipHostMallocDefault));
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    for (auto& e : ev_sub) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipEventCreateWithFlags(&ev_book, hipEventDisableTiming));
    return sync();
  }

  // Drain the stream; every staged upload has then been consumed.
  int sync() {
    HIPCHK(hipStreamSynchronize(stream));
    arena_used = 0;
    return MD_OK;
  }

  // GPU time between two events recorded on the stream (both complete).
  double elapsed_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
      (void)hipGetLastError();
      return 0.0;
    }
    return (double)ms;
  }

  // Stage host bytes in pinned memory and copy them to the device, in order on
  // the stream.  Small uploads take the next piece of the arena and do not
  // wait; the arena is recycled when the stream is drained (at the latest when
  // it is full).  Large uploads drain the stream and use the bulk stage.
  int upload(void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return MD_OK;
    const size_t need = (bytes + 255) & ~(size_t)255;
    if (need <= kArenaBytes) {
      if (arena_used + need > kArenaBytes) MDCHK(sync());
      std::memcpy(arena + arena_used, src, bytes);
      HIPCHK(hipMemcpyAsync(dst, arena + arena_used, bytes, hipMemcpyHostToDevice, stream));
      arena_used += need;
      return MD_OK;
    }
    MDCHK(sync());
    if (bytes > stage_cap) {
      if (no_alloc) return MD_ENOMEM;
      if (stage) (void)hipHostFree(stage);
      stage = nullptr;
      stage_cap = 0;
      HIPCHK(hipHostMalloc((void**)&stage, bytes, hipHostMallocDefault));
      stage_cap = bytes;
    }
    std::memcpy(stage, src, bytes);
    HIPCHK(hipMemcpyAsync(dst, stage, bytes, hipMemcpyHostToDevice, stream));
    return MD_OK;
  }

  // Upload unless dst already holds exactly these bytes from an earlier upload
  // (for descriptor arrays that only uploads write).
  int upload_cached(void* dst, const void* src, size_t bytes) {
    auto it = uploaded.find(dst);
    if (it != uploaded.end() && it->second.size() == bytes && std::memcmp(it->second.data(), src, bytes) == 0)
      return MD_OK;
    MDCHK(upload(dst, src, bytes));
    uploaded[dst].assign((const char*)src, (const char*)src + bytes);
    return MD_OK;
  }

  int ensure_stage(size_t bytes) {
    MDCHK(sync());
    if (bytes > stage_cap) {
      if (no_alloc) return MD_ENOMEM;
      if (stage) (void)hipHostFree(stage);
      stage = nullptr;
      stage_cap = 0;
      HIPCHK(hipHostMalloc((void**)&stage, bytes, hipHostMallocDefault));
      stage_cap = bytes;
    }
    return MD_OK;
  }

  // Bytes one step moves per particle of job h: x read and written, p read
  // and written, index, flag, count, the list (16-bit entries, kbar of them),
  // the tile's halo list, the noise cache read and written (FP32 class 12 +
  // 12, FP64 class 24 + 24), masses when they differ, and for bead models the
  // type and the inverse-permutation entries of the bonded partners.
  static double step_bytes_per_particle(const HostJob& h, double kbar) {
    double per = 105.0 + 2.0 * kbar + 6.0;
    if (h.dev.gamma > 0.0) per += h.dev.force_fp64 ? 48.0 : 24.0;
    if (!h.dev.uniform_mass) per += 8.0;
    if (h.model) per += 1.0 + 16.0;
    return per;
  }

  // Bytes one step moves for the resident jobs (the mean list length of the
  // last build; a guess of 12 before the first).
  double step_working_set() const {
    double ws = 0.0;
    for (int j = 0; j < max_jobs; ++j) {
      const HostJob& h = jobs[j];
      if (!h.used || h.n == 0) continue;
      const double kbar = h.nl_sum > 0.0 ? h.nl_sum / (double)h.n : 12.0;
      double per = step_bytes_per_particle(h, kbar);
      ws += (double)h.n * per;
    }
    return ws;
  }

  // Streaming stores for the new state (and list rows) when a step's data
  // exceed the 256 MB Infinity Cache of the MI355X (see the step kernel); the
  // kernel instances are chosen at launch, so cached graphs go when it flips.
  void set_store_policy() {
    const bool s = step_working_set() > kInfinityCacheBytes;
    if (s != stream_stores) {
      stream_stores = s;
      drop_graphs();
    }
  }

  // Job records in use: indices below this (the device copies of the job and
  // bookkeeping records are moved for these only; no kernel reads the others)
  int live_jobs() const {
    int n = 1;
    for (int j = 0; j < max_jobs; ++j)
      if (jobs[j].used) n = j + 1;
    return n;
  }

  int upload_jobs() {
    const int nj = live_jobs();
    std::vector<JobDev> tab(nj);
    for (int j = 0; j < nj; ++j) tab[j] = jobs[j].dev;
    return upload(B.jobs, tab.data(), sizeof(JobDev) * nj);
  }

  int read_book() {
    HIPCHK(hipMemcpyAsync(book_h, B.book, sizeof(JobBook) * live_jobs(), hipMemcpyDeviceToHost, stream));
    return sync();
  }

  static void tiles_of(const HostJob& h, int j, std::vector<int>& tj, std::vector<int64_t>& tf) {
    for (int64_t t = 0; t < h.n; t += kTile) {
      tj.push_back(j);
      tf.push_back(h.off + t);
    }
  }

  // ------------------------------------------------------------------ admission
  // Constants of a job with uniform mass d.mass (used when d.uniform_mass).
  static void mass_constants(JobDev& d) {
    const double m = d.mass > 0.0 ? d.mass : 1.0;
    d.noise_km = std::sqrt(m) * d.noise_k;
    d.dtm = d.dt / m;
    d.cpos = d.dt * d.dtm * 0.5;
    d.inv_cpos = 2.0 * m / (d.dt * d.dt);
  }

  static void fill_constants(HostJob& h) {
    const md_params& p = h.prm;
    JobDev& d = h.dev;
    d.dt = p.dt;
    d.half_dt = 0.5 * p.dt;
    d.gamma = p.gamma;
    d.b = 1.0 / (1.0 + 0.5 * p.dt * p.gamma);
    d.noise_k = p.gamma > 0.0 ? std::sqrt(2.0 * p.kT * p.gamma / p.dt) : 0.0;
    d.eps = p.eps;
    d.sig2 = p.sigma * p.sigma;
    d.pair_kind = p.pair_kind;
    const double rc = p.pair_kind != MD_PAIR_NONE ? p.rc : 0.0;
    const double skin = p.skin > 0.0 ? p.skin : 0.3;
    d.rc2 = rc * rc;
    const double rl = (rc > 0.0 ? rc : 1.0) + skin;
    d.rlist2 = rl * rl;
    // without a pair potential there are no lists to keep valid: no rebuilds
    d.half_skin = p.pair_kind != MD_PAIR_NONE ? 0.5 * skin : std::numeric_limits<double>::infinity();
    if (p.pair_kind != MD_PAIR_NONE) {
      double dphic;
      d.phic = lj_phi(p.eps, p.sigma, p.rc, &dphic);
      d.dphic = dphic;
    }
    d.force_fp64 = p.force_fp64 ? 1 : 0;
    d.newton_tol = p.newton_tol;
    // FP32-class exact sums: terms c dx stay below 2^19 while c < 2^19 / rc
    d.grid_bias = 0x1.8p20;
    d.grid_cmax = (float)(0x1p19 / (rc > 0.0 ? rc : 1.0) * (1.0 - 0x1p-10));
    mass_constants(d);
    d.newton_cap = p.newton_max_iter > 0 ? p.newton_max_iter : 32;
    d.newton_frozen = p.newton_frozen;
    d.model = h.model ? 1 : 0;
    d.bpm = h.model ? h.mdev.bpm : 0;
    d.seed = p.seed;
    d.surf_kind = h.surf_kind;
    for (int k = 0; k < MD_SURF_MAXPRM; ++k) d.surf[k] = h.surf[k];
    if (h.surf_kind == MD_SURF_ELLIPSOID)
      for (int k = 0; k < 3; ++k) d.surf[3 + k] = 1.0 / (h.surf[3 + k] * h.surf[3 + k]);
    if (h.surf_kind == MD_SURF_HEIGHT) {
      d.surf[2] = 2.0 / h.surf[2];
      d.surf[3] = 2.0 / h.surf[3];
    }
    if (h.surf_kind == MD_SURF_BRIDGE) {
      // device layout: x0 y0 z0, Lb/2, Rb, R, Rb + R, R/Rb
      d.surf[3] = 0.5 * h.surf[3];
      d.surf[6] = h.surf[4] + h.surf[5];
      d.surf[7] = h.surf[5] / h.surf[4];
    }
  }

  static int validate_particles(const HostJob& h, const double* x, const double* p, const double* mass,
                                const uint8_t* cons) {
    for (int64_t i = 0; i < h.n; ++i) {
      for (int k = 0; k < 3; ++k)
        if (!std::isfinite(x[3 * i + k]) || !std::isfinite(p[3 * i + k])) return MD_EINVAL;
      if (mass && !(mass[i] > 0.0)) return MD_EINVAL;
      const bool c = h.surf_kind != MD_SURF_NONE && (cons ? cons[i] != 0 : true);
      if (!c) continue;
      double n[3];
      const double g = host_g(h.surf_kind, h.surf, &x[3 * i], n);
      const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      if (!(nn > 0.0)) return MD_EOFFSURF;
      const double xs = std::max({1.0, std::fabs(x[3 * i]), std::fabs(x[3 * i + 1]), std::fabs(x[3 * i + 2])});
      const double ps =
          std::max({1.0, std::fabs(p[3 * i]), std::fabs(p[3 * i + 1]), std::fabs(p[3 * i + 2])});
      if (std::fabs(g) / nn > 1e-9 * xs) return MD_EOFFSURF;
      const double np = n[0] * p[3 * i] + n[1] * p[3 * i + 1] + n[2] * p[3 * i + 2];
      if (std::fabs(np) / nn > 1e-9 * ps) return MD_EOFFSURF;
    }
    return MD_OK;
  }

  static int64_t seg_slots(int64_t n) { return round_up(n + 1, kTile); }

  // Place a job: allocate its slots and bitmap words, upload its state.
  int admit(const md_params& prm, int surf_kind, const double* surf, int64_t n, const double* x,
            const double* p, const double* mass, const uint8_t* cons, const double* fcomb, int64_t step0,
            int64_t target, int* job_id, const ModelDev* model = nullptr, const uint8_t* types = nullptr) {
    MDCHK(validate_params(prm));
    // bead-model lists carry the partner type in the top two bits of a slot index
    if (model && (prm.pair_kind != MD_PAIR_LJ || (n > 0 && !types) || C > (int64_t)kIdMask))
      return MD_EINVAL;
    if (n < 0 || (n > 0 && (!x || !p)) || n > 0xFFFFFFF0LL) return MD_EINVAL;
    int j = -1;
    for (int q = 0; q < max_jobs; ++q)
      if (!jobs[q].used) {
        j = q;
        break;
      }
    if (j < 0) return MD_EAGAIN;
    HostJob h;
    h.used = true;
    h.prm = prm;
    h.surf_kind = surf_kind;
    for (int k = 0; k < MD_SURF_MAXPRM; ++k) h.surf[k] = surf ? surf[k] : 0.0;
    h.n = n;
    if (model) {
      h.model = true;
      h.mdev = *model;
    }
    fill_constants(h);
    MDCHK(validate_particles(h, x, p, mass, cons));
    MDCHK(make_grid(h, x));
    h.seg = seg_slots(n);
    h.off = slots.alloc(h.seg, kTile);
    if (h.off < 0) return MD_EAGAIN;
    h.bm_off = words.alloc(h.bm_words, 1);
    if (h.bm_off < 0) {
      slots.release(h.off, h.seg);
      return MD_EAGAIN;
    }
    JobDev& d = h.dev;
    d.off = h.off;
    d.n = n;
    d.bm_off = h.bm_off;
    d.xcur = d.pcur = d.scur = 0;
    d.step0 = step0;
    d.remaining = 0;
    d.mode = fcomb ? kModeStartGiven : kModeStart;
    bool uniform = true;
    double m0 = mass && n > 0 ? mass[0] : 1.0;
    if (mass)
      for (int64_t i = 1; i < n; ++i)
        if (mass[i] != m0) uniform = false;
    d.uniform_mass = uniform ? 1 : 0;
    d.mass = m0;
    d.inv_mass = 1.0 / m0;
    mass_constants(d);
    h.step = step0;
    h.target = target;
    h.last_build = step0;
    // upload: SoA positions, momenta, forces; ids in order; flags; masses
    if (n > 0) {
      // positions, momenta and forces are AoS on both sides: plain copies
      MDCHK(upload(B.X[0] + 3 * h.off, x, sizeof(double) * 3 * n));
      MDCHK(upload(B.P[0] + 3 * h.off, p, sizeof(double) * 3 * n));
      if (fcomb) MDCHK(upload(B.FC + 3 * h.off, fcomb, sizeof(double) * 3 * n));
      std::vector<uint32_t> ids(n);
      for (int64_t i = 0; i < n; ++i) ids[i] = (uint32_t)i;
      MDCHK(upload(B.ID[0] + h.off, ids.data(), sizeof(uint32_t) * n));
      std::vector<uint8_t> fl(n);
      for (int64_t i = 0; i < n; ++i) fl[i] = (surf_kind != MD_SURF_NONE && (cons ? cons[i] != 0 : true)) ? 1 : 0;
      MDCHK(upload(B.FLG[0] + h.off, fl.data(), n));
      for (int64_t i = 0; i < n; ++i) h.ndof += fl[i] ? 2.0 : 3.0;
      if (!uniform) MDCHK(upload(B.MASS[0] + h.off, mass, sizeof(double) * n));
      if (model) MDCHK(upload(B.TYPE[0] + h.off, types, n));
    }
    if (model) MDCHK(upload(const_cast<ModelDev*>(B.models) + j, model, sizeof(ModelDev)));
    jobs[j] = h;
    step_tiles_valid = false;
    *job_id = j;
    return MD_OK;
  }

  void drop(int j) {
    HostJob& h = jobs[j];
    if (!h.used) return;
    slots.release(h.off, h.seg);
    words.release(h.bm_off, h.bm_words);
    h = HostJob();
    step_tiles_valid = false;
  }

  // FP32-class step-kernel instance (kStepVariants); cached graphs hold the
  // old instance.
  void set_variant(int v) {
    v = std::max(0, std::min(kNumStepVariants - 1, v));
    if (v != f32_variant) {
      f32_variant = v;
      drop_graphs();
    }
  }

  // Counters plus the choices in effect.
  md_stats report() const {
    md_stats st = stats;
    st.step_variant = f32_variant;
    st.step_waves = kStepVariants[f32_variant].waves;
    st.step_halo_lds = kStepVariants[f32_variant].halo;
    st.list_capacity = kmax;
    st.skin = 0.0;
    st.reserved = 0.0;
    return st;
  }

  // Change a job's skin: new list radius and cell grid; the list is rebuilt
  // before the next step.
  int set_skin(int j, double skin) {
    HostJob& h = jobs[j];
    HostJob trial = h;
    trial.prm.skin = skin;
    fill_constants(trial);
    MDCHK(make_grid(trial, nullptr));
    if (trial.bm_words > h.bm_words) {
      words.release(h.bm_off, h.bm_words);
      const int64_t off = words.alloc(trial.bm_words, 1);
      if (off < 0) {
        const int64_t back = words.alloc(h.bm_words, 1);  // the freed segment is still there
        h.bm_off = back;
        return MD_ENOMEM;
      }
      trial.bm_off = off;
    } else {
      trial.bm_words = h.bm_words;  // keep the larger segment
    }
    trial.dev.bm_off = trial.bm_off;
    trial.built = false;
    trial.rate_prev = 0.0;
    h = trial;
    return MD_OK;
  }

  // ------------------------------------------------------------------ rebuild
  int grow_kmax(int need) {
    // whole rows, and only as large as needed: the list build holds the
    // lists of a tile in LDS
    const int nk = (std::max(need, kmax + kRow) + kRow - 1) / kRow * kRow;
    uint16_t* nl = nullptr;
    MDCHK(dalloc(&nl, (size_t)nk * C));
    // rows of entries k/8 do not move when rows are added
    HIPCHK(hipMemcpyAsync(nl, B.NL, sizeof(uint16_t) * (size_t)kmax * C, hipMemcpyDeviceToDevice, stream));
    MDCHK(sync());
    (void)hipFree(B.NL);
    B.NL = nl;
    kmax = nk;
    B.kmax = nk;
    nl_bytes = (size_t)nk * C * 2;
    drop_graphs();
    return MD_OK;
  }

  // A larger halo capacity per tile (the lists are built again afterwards).
  int grow_hcap(int need) {
    if (need > kMaxHcap) return MD_ENOMEM;
    int nh = std::min(kMaxHcap, std::max(need + need / 4, hcap + 64));
    nh = std::min(kMaxHcap, (nh + 63) / 64 * 64);
    uint32_t* hl = nullptr;
    MDCHK(sync());
    MDCHK(dalloc(&hl, (size_t)(C / kTile + 1) * nh));
    (void)hipFree(B.HALO);
    B.HALO = hl;
    hcap = nh;
    B.hcap = nh;
    drop_graphs();
    return MD_OK;
  }

  // Sort the jobs of `set` into cell order and build their neighbour lists.
  // Nothing here waits for the device: the list statistics (and an overflow
  // of the list capacity, which also stops the job before its first step on
  // the new lists) are read back with the job records after the next chunk.
  int rebuild(const std::vector<int>& set) {
    if (set.empty()) return MD_OK;
    std::vector<int> tj;
    std::vector<int64_t> tf;
    std::vector<Chunk> cb, cc;
    std::vector<Range> rb, rcnt;
    std::vector<Range> rtacc;
    int64_t seg_chunks_max = 0;  // chunks of the longest scan segment
    for (int j : set) {
      HostJob& h = jobs[j];
      h.dev.remaining = 0;
      h.dev.step0 = h.step;
      tiles_of(h, j, tj, tf);
      rb.push_back({h.bm_off, h.bm_words});
      rcnt.push_back({h.off, h.n + 1});
      rtacc.push_back({2 * (h.off / kGroup), 2 * ((h.n + kGroup - 1) / kGroup)});  // doubles as word pairs
      int first = (int)cb.size();
      for (int64_t s = 0; s < h.bm_words; s += kScanChunk)
        cb.push_back({h.bm_off + s, (int)std::min<int64_t>(kScanChunk, h.bm_words - s), first});
      seg_chunks_max = std::max<int64_t>(seg_chunks_max, (int64_t)cb.size() - first);
      first = (int)cc.size();
      for (int64_t s = 0; s < h.n + 1; s += kScanChunk)
        cc.push_back({h.off + s, (int)std::min<int64_t>(kScanChunk, h.n + 1 - s), first});
      seg_chunks_max = std::max<int64_t>(seg_chunks_max, (int64_t)cc.size() - first);
    }
    if (tj.empty()) {
      // only empty jobs: nothing to sort; their records start afresh
      for (int j : set) {
        jobs[j].built = true;
        jobs[j].A_now = 0.0;
        book_h[j] = fresh_book();
        HIPCHK(hipMemcpyAsync(&B.book[j], &book_h[j], sizeof(JobBook), hipMemcpyHostToDevice, stream));
      }
      return MD_OK;
    }
    if ((int64_t)(cb.size() + cc.size()) > chunk_cap || (int64_t)tj.size() > tile_cap ||
        (int64_t)(rb.size() + rcnt.size() + rtacc.size()) > range_cap)
      return MD_ENOMEM;
    bool wide = false;  // FP64-class or bead-model jobs among those built
    for (int j : set) wide = wide || jobs[j].dev.force_fp64 || jobs[j].model;
    // the wide instance's table of window records: in LDS when it fits
    const int64_t wlen = (int64_t)kTile + hcap;
    size_t lds = nlist_lds_bytes(kmax, wide ? wlen : 0);
    B.KKEY = nullptr;
    if (wide && (list_table_global || (int64_t)lds + nlist_static_lds(wide) > (int64_t)lds_max)) {
      lds = nlist_lds_bytes(kmax, 0);
      const int64_t need = (int64_t)tj.size() * wlen;
      if (need > kkey_cap) {
        if (kkey_d) (void)hipFree(kkey_d);
        kkey_d = nullptr;
        kkey_cap = 0;
        MDCHK(dalloc(&kkey_d, (size_t)need));
        kkey_cap = need;
      }
      B.KKEY = kkey_d;
    }
    if ((int64_t)lds + nlist_static_lds(wide) > (int64_t)lds_max) return MD_ENOMEM;
    MDCHK(upload_jobs());
    MDCHK(upload_cached(aux_tiles_job, tj.data(), sizeof(int) * tj.size()));
    MDCHK(upload_cached(aux_tiles_first, tf.data(), sizeof(int64_t) * tf.size()));
    std::vector<Chunk> call(cb);
    call.insert(call.end(), cc.begin(), cc.end());
    // seg_first stays relative to each sub-list: the two scans get separate base pointers
    MDCHK(upload_cached(chunks_d, call.data(), sizeof(Chunk) * call.size()));
    std::vector<Range> rall(rb);
    rall.insert(rall.end(), rcnt.begin(), rcnt.end());
    rall.insert(rall.end(), rtacc.begin(), rtacc.end());
    MDCHK(upload_cached(ranges_d, rall.data(), sizeof(Range) * rall.size()));
    const int ntiles = (int)tj.size();
    if (!build_timing_pending) HIPCHK(hipEventRecord(ev[2], stream));
    // zero bitmaps and cell counters
    {
      // one launch for the three sets of ranges; fewer workgroups per range
      // when there are many ranges
      const int nr = (int)rall.size();
      const int gx = std::max(4, std::min(256, 4096 / std::max(1, nr)));
      for (int q0 = 0; q0 < nr; q0 += 65535)  // the grid's y extent is at most 65535
        hipLaunchKernelGGL(k_zero_ranges, dim3(gx, (unsigned)std::min(65535, nr - q0)), dim3(256), 0, stream, B.BM,
                           B.CCNT, (uint32_t*)B.TACC, ranges_d, (int)rb.size(), (int)rcnt.size(), q0);
    }
    // k_mark resets the job records of jobs with particles; the others are reset here
    for (int j : set) {
      if (jobs[j].n > 0) continue;
      book_h[j] = fresh_book();
      HIPCHK(hipMemcpyAsync(&B.book[j], &book_h[j], sizeof(JobBook), hipMemcpyHostToDevice, stream));
    }
    hipLaunchKernelGGL(k_mark, dim3(ntiles), dim3(kTile), 0, stream, B, aux_tiles_job, aux_tiles_first);
    // bitmap popcount prefix (segmented by job)
    const int nb = (int)cb.size(), nc = (int)cc.size();
    // segments of few chunks: passes B and C in one launch
    const bool bc = seg_chunks_max <= kScanBcMax && !scan_three_pass;
    auto scan_rest = [&](uint32_t* out, const Chunk* ch, uint32_t* sums, int n) {
      if (bc) {
        hipLaunchKernelGGL(k_scan_bc, dim3(n), dim3(kScanThreads), 0, stream, out, ch, sums);
      } else {
        hipLaunchKernelGGL(k_scan_b, dim3(1), dim3(kScanB), 0, stream, sums, ch, n);
        hipLaunchKernelGGL(k_scan_c, dim3(n), dim3(kScanThreads), 0, stream, out, ch, sums);
      }
    };
    hipLaunchKernelGGL(k_scan_a<true>, dim3(nb), dim3(kScanThreads), 0, stream, B.BM, B.WOFF, chunks_d, chunk_sums);
    scan_rest(B.WOFF, chunks_d, chunk_sums, nb);
    hipLaunchKernelGGL(k_count, dim3(ntiles), dim3(kTile), 0, stream, B, aux_tiles_job, aux_tiles_first);
    // cell starts (segmented by job)
    hipLaunchKernelGGL(k_scan_a<false>, dim3(nc), dim3(kScanThreads), 0, stream, B.CCNT, B.CSTART, chunks_d + nb,
                       chunk_sums + nb);
    scan_rest(B.CSTART, chunks_d + nb, chunk_sums + nb, nc);
    hipLaunchKernelGGL(k_move, dim3(ntiles), dim3(kTile), 0, stream, B, aux_tiles_job, aux_tiles_first);
    set_store_policy();
    const dim3 ng(ntiles), nb_(kNlistBlock);
    if (wide && stream_stores)
      hipLaunchKernelGGL((k_nlist<true, true>), ng, nb_, lds, stream, B, B.jobs, B.models, aux_tiles_job, aux_tiles_first);
    else if (wide)
      hipLaunchKernelGGL((k_nlist<true, false>), ng, nb_, lds, stream, B, B.jobs, B.models, aux_tiles_job, aux_tiles_first);
    else if (stream_stores)
      hipLaunchKernelGGL((k_nlist<false, true>), ng, nb_, lds, stream, B, B.jobs, B.models, aux_tiles_job, aux_tiles_first);
    else
      hipLaunchKernelGGL((k_nlist<false, false>), ng, nb_, lds, stream, B, B.jobs, B.models, aux_tiles_job, aux_tiles_first);
    hipLaunchKernelGGL(k_job_stats, dim3(live_jobs()), dim3(kStatsThreads), 0, stream, B, 1);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(ev[3], stream));
    build_timing_pending = true;
    stats.builds += 1;
    for (int j : set) {
      HostJob& h = jobs[j];
      h.dev.xcur ^= 1;
      h.dev.pcur ^= 1;
      h.dev.scur ^= 1;
      h.built = true;
      h.breach_base = h.sum_breaches;  // the build starts the device counter afresh
      h.lists_pending = true;
      if (h.step > h.last_build && h.A_now > 0.0) h.rate_prev = h.A_now / (double)(h.step - h.last_build);
      h.A_now = 0.0;
      h.last_build = h.step;
      h.rebuilds += 1;
    }
    return MD_OK;
  }

  // After a drained stream: take the list statistics of the last builds from
  // the job records in book_h, and the build time.  Returns the largest list
  // length found (for a capacity check).
  // Also grows the halo capacity when a tile's halo did not fit (the jobs
  // concerned were stopped before their first step and are built again), and
  // fails the jobs whose neighbourhoods the staged build could not hold.
  int collect_build_stats(int* halo_need = nullptr) {
    if (build_timing_pending) {
      stats.rebuild_ms += elapsed_ms(ev[2], ev[3]);
      build_timing_pending = false;
    }
    int need = 0, hneed = 0;
    double sum = 0.0, cnt = 0.0;
    for (int j = 0; j < max_jobs; ++j) {
      HostJob& h = jobs[j];
      if (!h.used || !h.lists_pending) continue;
      h.lists_pending = false;
      if (h.n == 0) continue;
      h.nl_max = book_h[j].nl_max;
      h.nl_sum = book_h[j].nl_sum;
      h.halo_max = book_h[j].halo_max;
      if (book_h[j].build_fail) {
        h.status = MD_ENOMEM;
        h.done = true;
        step_tiles_valid = false;
        continue;
      }
      need = std::max(need, h.nl_max);
      hneed = std::max(hneed, h.halo_max);
      sum += h.nl_sum;
      cnt += (double)h.n;
    }
    if (cnt > 0) stats.nl_mean = sum / cnt;
    if (halo_need) *halo_need = hneed;
    return need;
  }

  // Build the lists of `set` and wait for them; on a capacity overflow grow the
  // capacity and build again (for callers that use the lists at once).
  int rebuild_now(const std::vector<int>& set) {
    for (int attempt = 0; attempt < 6; ++attempt) {
      MDCHK(rebuild(set));
      MDCHK(read_book());
      int hneed = 0;
      const int need = collect_build_stats(&hneed);
      if (need <= kmax && hneed <= hcap) return MD_OK;
      if (need > kmax) MDCHK(grow_kmax(need + need / 8 + 2));
      if (hneed > hcap) MDCHK(grow_hcap(hneed));
      for (int j : set) jobs[j].built = false;
    }
    return MD_ENOMEM;
  }

  // ------------------------------------------------------------------ stepping
  bool steppable(const HostJob& h) const { return h.used && h.status == MD_OK && !h.done && h.step < h.target; }

  static int grid_for(int count) {
    if (count <= 0) return 0;
    int g = 64;
    while (g < count) g *= 2;
    return g;
  }

  static int class_of(const HostJob& h) {
    return (h.model ? 2 : 0) + (h.dev.force_fp64 ? 0 : 1) + (heavy_surface(h.surf_kind) ? 4 : 0);
  }

  // Upload the tile lists of the steppable jobs.  Graphs bake the grid size,
  // not the lists: they stay valid while each list fits its grid and is not
  // much smaller than it.
  int prepare_step_tiles() {
    if (step_tiles_valid) return MD_OK;
    std::vector<int> tj[kClasses];
    std::vector<int64_t> tf[kClasses];
    for (int j = 0; j < max_jobs; ++j) {
      const HostJob& h = jobs[j];
      if (!h.used || h.done || h.status != MD_OK) continue;
      tiles_of(h, j, tj[class_of(h)], tf[class_of(h)]);
    }
    bool same = true;
    for (int c = 0; c < kClasses; ++c) {
      if ((int64_t)tj[c].size() > tile_cap) return MD_ENOMEM;
      same = same && tj[c] == last_tj[c] && tf[c] == last_tf[c];
    }
    step_tiles_valid = true;
    if (same) return MD_OK;
    int counts[kClasses];
    for (int c = 0; c < kClasses; ++c) {
      counts[c] = (int)tj[c].size();
      if (!tj[c].empty()) {
        MDCHK(upload(step_tiles_job + c * tile_cap, tj[c].data(), sizeof(int) * tj[c].size()));
        MDCHK(upload(step_tiles_first + c * tile_cap, tf[c].data(), sizeof(int64_t) * tf[c].size()));
      }
      last_tj[c].swap(tj[c]);
      last_tf[c].swap(tf[c]);
    }
    MDCHK(upload(step_counts, counts, sizeof(counts)));
    auto fits = [](int g, int count, int want) {
      if (count == 0) return g == 0;
      return g >= count && g <= 4 * want;
    };
    bool refit = false;
    for (int c = 0; c < kClasses; ++c) refit = refit || !fits(grid[c], counts[c], grid_for(counts[c]));
    if (refit) {
      for (int c = 0; c < kClasses; ++c) grid[c] = grid_for(counts[c]);
      drop_graphs();
    }
    return MD_OK;
  }

  // One step launch of tile class c (see class_of) on stream s.
  void launch_class(int c, int t, bool stream_st, hipStream_t s) {
    const StepLaunch L{dim3(grid[c]), s, &B, step_tiles_job + c * tile_cap, step_tiles_first + c * tile_cap,
                       step_counts + c, t};
    const bool all = c >= 4;
    switch (c & 3) {
      case 0: launch_step_f64(L, all, stream_st); break;
      case 1: launch_step_f32(L, f32_variant, all, stream_st); break;
      case 2: launch_step_model(L, true, all, stream_st); break;
      default: launch_step_model(L, false, all, stream_st); break;
    }
  }

  void enqueue_steps_as(int t0, int k, bool stream_st, hipStream_t s) {
    for (int t = t0; t < t0 + k; ++t)
      for (int c = 0; c < kClasses; ++c)
        if (grid[c] > 0) launch_class(c, t, stream_st, s);
  }

  void enqueue_steps(int t0, int k) { enqueue_steps_as(t0, k, stream_stores, stream); }

  // The graph of steps t = 0 .. k-1 under the current tile grids and store
  // policy, captured on stream s when it is not cached (capture only records
  // the launches: s may be a stream that never runs them).
  int step_graph(int k, hipStream_t s, hipGraphExec_t* out) {
    auto it = graphs.find(GraphKey{k});
    if (it == graphs.end()) {
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      enqueue_steps_as(0, k, stream_stores, s);
      HIPCHK(hipStreamEndCapture(s, &g));
      hipGraphExec_t ex = nullptr;
      const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPCHK(e);
      it = graphs.emplace(GraphKey{k}, ex).first;
    }
    *out = it->second;
    return MD_OK;
  }

  int launch_chunk(int k, bool use_graph) {
    if (!use_graph) {
      enqueue_steps(0, k);
      HIPCHK(hipGetLastError());
      return MD_OK;
    }
    hipGraphExec_t ex = nullptr;
    MDCHK(step_graph(k, stream, &ex));
    HIPCHK(hipGraphLaunch(ex, stream));
    return MD_OK;
  }

  // Steps a job can take before its list goes stale: the remaining half skin
  // over the larger of the displacement rates of this and the previous list.
  // A list that goes stale earlier stops its job on the device, so the
  // estimate need not be conservative.
  static int predict_chunk(const HostJob& h) {
    const int64_t since = h.step - h.last_build;
    double rate = h.rate_prev;
    if (since > 0 && h.A_now > 0.0) rate = std::max(rate, h.A_now / (double)since);
    if (!(rate > 0.0)) return 16;
    const double left = (h.dev.half_skin - h.A_now) / rate;
    return (int)std::max(0.0, std::min(1e6, std::floor(left)));
  }

  // One chunk of at most kcap steps for every steppable job; rebuilds first
  // where a list is missing or would go stale within the chunk.
  // eager = true (pools): rebuild every job whose list would go stale within
  // the chunk, and run the full chunk; eager = false (one system): rebuild only
  // when the list is (nearly) stale and shorten the chunk to the prediction.
  // A chunk of k steps is one graph of k steps with one upload of the job
  // records before it, once that graph is cached; until then a run of cached
  // graphs of power-of-two lengths (the binary digits of k), with the job
  // records for each uploaded before it, while the graph of k steps is
  // captured on a side stream.  The host waits once, for the job records at
  // the end.
  int run_chunk(int kcap, bool use_graph, int64_t* advanced, bool eager = false) {
    MDCHK(enqueue_chunk(kcap, use_graph, eager));
    return complete_chunk(advanced);
  }

  // The first half of run_chunk: rebuilds, the chunk's graphs and the copy of
  // the job records to the host are enqueued, and the call returns without
  // waiting (complete_chunk waits).  Until then the host may admit jobs: their
  // uploads go to slots the chunk does not touch and follow it on the stream.
  int enqueue_chunk(int kcap, bool use_graph, bool eager) {
    inflight.active = false;
    std::vector<int> need;
    const int k = std::min(kcap, kMaxChunk);
    for (int j = 0; j < max_jobs; ++j) {
      HostJob& h = jobs[j];
      if (!steppable(h)) continue;
      if (!h.built) {
        need.push_back(j);
        continue;
      }
      const int pk = predict_chunk(h);
      if (pk < (eager ? std::min<int64_t>(k, h.target - h.step) : 2)) need.push_back(j);
    }
    MDCHK(rebuild(need));
    int kk = k;
    bool any = false;
    for (int j = 0; j < max_jobs; ++j) {
      HostJob& h = jobs[j];
      if (!steppable(h)) continue;
      any = true;
      if (!eager) kk = std::min<int64_t>(kk, std::max(1, predict_chunk(h)));
    }
    if (!any) return MD_OK;
    std::vector<int64_t>& cap = inflight.cap;
    cap.assign(max_jobs, 0);
    for (int j = 0; j < max_jobs; ++j) {
      HostJob& h = jobs[j];
      cap[j] = steppable(h) ? std::min<int64_t>(h.target - h.step, kk) : 0;
      h.dev.step0 = h.step;
      h.dev.remaining = cap[j];
    }
    MDCHK(prepare_step_tiles());
    set_store_policy();
    const int nj = live_jobs();
    std::vector<JobDev> tab(nj);
    int nsub = 0;
    // sub-chunk [t0, t0 + len): the job records for it, then its launches
    auto sub_chunk = [&](int t0, int len, bool graph) -> int {
      for (int j = 0; j < nj; ++j) {
        const HostJob& h = jobs[j];
        JobDev d = h.dev;
        d.step0 = h.step + t0;
        d.remaining = std::max<int64_t>(0, std::min<int64_t>(cap[j] - t0, len));
        d.xcur = h.dev.xcur ^ (t0 & 1);
        if (t0 > 0) d.mode = kModeSteady;
        tab[j] = d;
      }
      MDCHK(upload(B.jobs, tab.data(), sizeof(JobDev) * nj));
      HIPCHK(hipEventRecord(ev_sub[2 * nsub], stream));
      MDCHK(launch_chunk(len, graph));
      HIPCHK(hipEventRecord(ev_sub[2 * nsub + 1], stream));
      ++nsub;
      return MD_OK;
    };
    if (!use_graph || graphs.count(GraphKey{kk})) {
      // one launch sequence (or the chunk's own cached graph)
      MDCHK(sub_chunk(0, kk, use_graph));
    } else {
      // the cached graphs of power-of-two lengths (the binary digits of kk,
      // each with its job records); then, while they run, the graph of the
      // whole chunk is captured on a side stream for the next chunk of kk steps
      int t0 = 0;
      for (int len = kMaxChunk; len >= 1; len >>= 1) {
        if (!(kk & len)) continue;
        MDCHK(sub_chunk(t0, len, true));
        t0 += len;
      }
      if (nsub > 1) {
        hipGraphExec_t ex = nullptr;
        MDCHK(step_graph(kk, cap_stream, &ex));
      }
    }
    hipLaunchKernelGGL(k_job_stats, dim3(nj), dim3(kStatsThreads), 0, stream, B, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(book_h, B.book, sizeof(JobBook) * nj, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipEventRecord(ev_book, stream));
    int classes = 0;
    for (int c = 0; c < kClasses; ++c) classes += grid[c] > 0;
    inflight.kk = kk;
    inflight.nsub = nsub;
    inflight.launches = (int64_t)kk * classes;
    inflight.active = true;
    return MD_OK;
  }

  // The second half: wait for the job records of the chunk in flight and
  // advance the jobs' steps from them.
  int complete_chunk(int64_t* advanced) {
    *advanced = 0;
    if (!inflight.active) return MD_OK;
    inflight.active = false;
    HIPCHK(hipEventSynchronize(ev_book));
    const std::vector<int64_t>& cap = inflight.cap;
    const int nsub = inflight.nsub;
    for (int q = 0; q < nsub; ++q) stats.step_kernel_ms += elapsed_ms(ev_sub[2 * q], ev_sub[2 * q + 1]);
    stats.chunks += 1;
    stats.step_launches += inflight.launches;
    int halo_need = 0;
    const int longest = collect_build_stats(&halo_need);
    int64_t adv = 0;
    for (int j = 0; j < max_jobs; ++j) {
      HostJob& h = jobs[j];
      if (!h.used || cap[j] == 0) continue;
      const JobBook& K = book_h[j];
      int64_t done = cap[j];
      if (K.stop_at < h.step + done) done = std::max<int64_t>(0, K.stop_at - h.step);
      h.newton_max = std::max(h.newton_max, K.newton_max);
      h.sum_breaches = h.breach_base + K.sum_breaches;
      if (K.err_key != kNoError) {
        // the launch of step err_step failed: the state is that after it (its
        // position stage ran), undefined for the failing particles
        h.status = (int)(K.err_key & 3u) == kErrNewton ? MD_ENEWTON : MD_ENAN;
        h.err_id = (int)(K.err_key >> 2);
        h.err_step = K.err_step;
        if (done & 1) h.dev.xcur ^= 1;
        h.step += done;
        h.done = true;
        step_tiles_valid = false;
        stats.steps += done;
        stats.particle_steps += done * h.n;
        continue;
      }
      h.step += done;
      if (done & 1) h.dev.xcur ^= 1;
      if (done > 0) h.dev.mode = kModeSteady;
      h.A_now = K.a_now;
      // a stale list, or one that overflowed its capacity, is built again
      if (K.stop_at != kNever || h.A_now > h.dev.half_skin) h.built = false;
      if (h.step >= h.target) {
        h.done = true;
        step_tiles_valid = false;
      }
      adv = std::max<int64_t>(adv, done);
      stats.steps += done;
      stats.particle_steps += done * h.n;
    }
    if (longest > kmax) MDCHK(grow_kmax(longest + longest / 8 + 2));
    if (halo_need > hcap) MDCHK(grow_hcap(halo_need));
    *advanced = adv;
    return MD_OK;
  }

  // Complete the chunk in flight, if any (before anything that reads or
  // frees device state of the jobs).
  int drain() {
    int64_t adv = 0;
    return complete_chunk(&adv);
  }

  // ------------------------------------------------------------------ finish
  // State at the current step by particle index.  dev: x, p, f are device
  // pointers (filled by device-to-device copies on the library's stream),
  // else host pointers; any may be NULL.
  // noalloc (with dev): the reduction works in `scratch` and the four results
  // come back through the pinned arena; no device or pinned host memory is
  // allocated (a list build that would need more capacity fails with
  // MD_ENOMEM instead of growing it).
  int finish(int j, double* x, double* p, double* f, md_diag* diag, bool dev = false, bool noalloc = false) {
    HostJob& h = jobs[j];
    if (!h.used) return MD_ENOTFOUND;
    if (h.n == 0) {
      // (the counters as finish_many reports them)
      if (diag) {
        std::memset(diag, 0, sizeof(*diag));
        diag->step = h.step;
        diag->rebuilds = h.rebuilds;
        diag->newton_iter_max = h.newton_max;
        diag->nlist_max = h.nl_max;
        diag->error_index = -1;
        diag->error_step = -1;
        diag->exact_sum_breaches = h.sum_breaches;
      }
      return h.status;
    }
    if (h.status == MD_OK && (!h.built || h.A_now > h.dev.half_skin)) MDCHK(rebuild_now({j}));
    h.dev.step0 = h.step;
    h.dev.remaining = 0;
    MDCHK(upload_jobs());
    std::vector<int> tj;
    std::vector<int64_t> tf;
    tiles_of(h, j, tj, tf);
    MDCHK(upload_cached(aux_tiles_job, tj.data(), sizeof(int) * tj.size()));
    MDCHK(upload_cached(aux_tiles_first, tf.data(), sizeof(int64_t) * tf.size()));
    if (h.dev.force_fp64)
      hipLaunchKernelGGL(k_finish<true>, dim3((unsigned)tj.size()), dim3(kTile), 0, stream, B, aux_tiles_job,
                         aux_tiles_first);
    else
      hipLaunchKernelGGL(k_finish<false>, dim3((unsigned)tj.size()), dim3(kTile), 0, stream, B, aux_tiles_job,
                         aux_tiles_first);
    const int64_t n = h.n;
    const int nb = (int)std::min<int64_t>(kDiagBlocks, (n + kDiagThreads - 1) / kDiagThreads);
    double* part = noalloc ? scratch_d : diag_d;
    if (nb > kDiagBlocks) return MD_EINVAL;  // the partials would not fit `scratch` (cannot happen: nb is capped)
    hipLaunchKernelGGL(k_diag_partial, dim3(nb), dim3(kDiagThreads), 0, stream, B.OD, (int64_t)C, h.off, n, part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagThreads), 0, stream, part, nb, part + 4 * kDiagBlocks);
    HIPCHK(hipGetLastError());
    const size_t vb = sizeof(double) * 3 * n;
    double* st = nullptr;  // host copies (host variant) and the four results
    double* red_h = nullptr;
    if (noalloc) {
      if (arena_used + 256 > kArenaBytes) MDCHK(sync());
      red_h = (double*)(arena + arena_used);
      arena_used += 256;
    } else {
      MDCHK(ensure_stage(3 * vb + 4 * sizeof(double)));
      st = (double*)stage;
      red_h = st + 9 * n;
    }
    const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    double* dst[3] = {dev ? x : st, dev ? p : st + 3 * n, dev ? f : st + 6 * n};
    const double* src[3] = {B.OX + 3 * h.off, B.OP + 3 * h.off, B.OF + 3 * h.off};
    const bool want[3] = {x != nullptr, p != nullptr, f != nullptr};
    for (int k = 0; k < 3; ++k)
      if (want[k]) HIPCHK(hipMemcpyAsync(dst[k], src[k], vb, kind, stream));
    HIPCHK(hipMemcpyAsync(red_h, part + 4 * kDiagBlocks, 4 * sizeof(double), hipMemcpyDeviceToHost, stream));
    MDCHK(sync());
    if (!dev) {
      if (x) std::memcpy(x, st, vb);
      if (p) std::memcpy(p, st + 3 * n, vb);
      if (f) std::memcpy(f, st + 6 * n, vb);
    }
    if (diag) {
      const double* red = red_h;
      const double K = red[0], U = red[1], gd = red[2], nv = red[3], ndof = h.ndof;
      std::memset(diag, 0, sizeof(*diag));
      diag->K = K;
      diag->U = U;
      diag->ndof = ndof;
      diag->kT = ndof > 0 ? 2.0 * K / ndof : 0.0;
      diag->gdist_max = gd;
      diag->nv_max = nv;
      diag->step = h.step;
      diag->rebuilds = h.rebuilds;
      diag->newton_iter_max = h.newton_max;
      diag->nlist_max = h.nl_max;
      diag->error_index = h.err_id;
      diag->error_step = h.err_step;
      diag->exact_sum_breaches = h.sum_breaches;
    }
    return h.status;
  }

  // finish() for several jobs into host arrays: one list build for the jobs
  // whose lists are stale, the finish and diagnostics kernels and copies of
  // every job enqueued back to back, and one wait.  status[q] receives job
  // ids[q]'s own status (or MD_ENOTFOUND).
  int finish_many(const int* ids, int n, double* const* xs, double* const* ps, md_diag* diags, int* status) {
    std::vector<int> need;
    for (int q = 0; q < n; ++q) {
      const int j = ids[q];
      if (j < 0 || j >= max_jobs || !jobs[j].used) continue;
      const HostJob& h = jobs[j];
      if (h.n > 0 && h.status == MD_OK && (!h.built || h.A_now > h.dev.half_skin)) need.push_back(j);
    }
    if (!need.empty()) MDCHK(rebuild_now(need));
    size_t bytes = 4 * sizeof(double) * (size_t)n;
    std::vector<size_t> at(n, 0);
    for (int q = 0; q < n; ++q) {
      const int j = ids[q];
      if (j < 0 || j >= max_jobs || !jobs[j].used) continue;
      HostJob& h = jobs[j];
      h.dev.step0 = h.step;
      h.dev.remaining = 0;
      at[q] = bytes;
      bytes += 2 * sizeof(double) * 3 * (size_t)h.n;
    }
    // device buffers: the jobs' diagnostic partials, the packed results
    // (diagnostics, then each job's x and p, as laid out by `at`) and the two
    // job tables
    if ((int64_t)n * 4 * kDiagBlocks > diag_many_cap) {
      if (diag_many) (void)hipFree(diag_many);
      diag_many = nullptr;
      diag_many_cap = 0;
      MDCHK(dalloc(&diag_many, (size_t)n * 4 * kDiagBlocks));
      diag_many_cap = (int64_t)n * 4 * kDiagBlocks;
    }
    const int64_t pack_doubles = (int64_t)(bytes / sizeof(double));
    if (pack_doubles > pack_cap) {
      if (pack_d) (void)hipFree(pack_d);
      pack_d = nullptr;
      pack_cap = 0;
      MDCHK(dalloc(&pack_d, (size_t)pack_doubles));
      pack_cap = pack_doubles;
    }
    const size_t tab_bytes = (sizeof(DiagJob) + sizeof(PackJob)) * (size_t)n;
    if ((int64_t)tab_bytes > fj_cap) {
      if (fj_d) (void)hipFree(fj_d);
      fj_d = nullptr;
      fj_cap = 0;
      MDCHK(dalloc(&fj_d, tab_bytes));
      fj_cap = (int64_t)tab_bytes;
    }
    MDCHK(ensure_stage(bytes));  // (waits for the stream)
    MDCHK(upload_jobs());
    char* st = (char*)stage;
    // all the fetched jobs at once: one finish launch per force class over
    // their tiles (FP64 class first), one pair of diagnostic launches, one
    // packing launch and one copy to the host
    std::vector<int> tj, tj32;
    std::vector<int64_t> tf, tf32;
    std::vector<char> tabs(tab_bytes);
    DiagJob* djs = reinterpret_cast<DiagJob*>(tabs.data());
    PackJob* pjs = reinterpret_cast<PackJob*>(tabs.data() + sizeof(DiagJob) * (size_t)n);
    int64_t maxn = 0;
    for (int q = 0; q < n; ++q) {
      const int j = ids[q];
      const bool ok = j >= 0 && j < max_jobs && jobs[j].used && jobs[j].n > 0;
      const HostJob* h = ok ? &jobs[j] : nullptr;
      const int64_t nq = ok ? h->n : 0;
      djs[q] = DiagJob{ok ? h->off : 0, nq, std::min<int64_t>(kDiagBlocks, (nq + kDiagThreads - 1) / kDiagThreads)};
      pjs[q] = PackJob{ok ? h->off : 0, nq, (int64_t)(at[q] / sizeof(double))};
      maxn = std::max(maxn, nq);
      if (ok) {
        if (h->dev.force_fp64)
          tiles_of(*h, j, tj, tf);
        else
          tiles_of(*h, j, tj32, tf32);
      }
    }
    const int n64 = (int)tj.size(), n32 = (int)tj32.size();
    tj.insert(tj.end(), tj32.begin(), tj32.end());
    tf.insert(tf.end(), tf32.begin(), tf32.end());
    if (!tj.empty()) {
      MDCHK(upload_cached(aux_tiles_job, tj.data(), sizeof(int) * tj.size()));
      MDCHK(upload_cached(aux_tiles_first, tf.data(), sizeof(int64_t) * tf.size()));
    }
    if (n64 > 0)
      hipLaunchKernelGGL(k_finish<true>, dim3((unsigned)n64), dim3(kTile), 0, stream, B, aux_tiles_job,
                         aux_tiles_first);
    if (n32 > 0)
      hipLaunchKernelGGL(k_finish<false>, dim3((unsigned)n32), dim3(kTile), 0, stream, B, aux_tiles_job + n64,
                         aux_tiles_first + n64);
    MDCHK(upload(fj_d, tabs.data(), tab_bytes));
    const DiagJob* dj_d = reinterpret_cast<const DiagJob*>(fj_d);
    const PackJob* pj_d = reinterpret_cast<const PackJob*>(fj_d + sizeof(DiagJob) * (size_t)n);
    const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (3 * maxn + 255) / 256));
    for (int q0 = 0; q0 < n; q0 += 65535) {  // the grid's y extent is at most 65535
      const unsigned ny = (unsigned)std::min(65535, n - q0);
      hipLaunchKernelGGL(k_diag_partial_many, dim3(kDiagBlocks, ny), dim3(kDiagThreads), 0, stream, B.OD, (int64_t)C,
                         dj_d, q0, diag_many);
      hipLaunchKernelGGL(k_pack_xp, dim3(gx, ny), dim3(256), 0, stream, B.OX, B.OP, pj_d, q0, pack_d);
    }
    hipLaunchKernelGGL(k_diag_final_many, dim3((unsigned)n), dim3(kDiagThreads), 0, stream, diag_many, dj_d, pack_d);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(st, pack_d, bytes, hipMemcpyDeviceToHost, stream));
    MDCHK(sync());
    for (int q = 0; q < n; ++q) {
      const int j = ids[q];
      if (j < 0 || j >= max_jobs || !jobs[j].used) {
        if (status) status[q] = MD_ENOTFOUND;
        continue;
      }
      const HostJob& h = jobs[j];
      const size_t vb = sizeof(double) * 3 * (size_t)h.n;
      if (h.n > 0) {
        if (xs && xs[q]) std::memcpy(xs[q], st + at[q], vb);
        if (ps && ps[q]) std::memcpy(ps[q], st + at[q] + vb, vb);
      }
      if (diags) {
        md_diag& d = diags[q];
        std::memset(&d, 0, sizeof(d));
        const double* red = (const double*)st + 4 * q;
        if (h.n > 0) {
          d.K = red[0];
          d.U = red[1];
          d.gdist_max = red[2];
          d.nv_max = red[3];
        }
        d.ndof = h.ndof;
        d.kT = h.ndof > 0 ? 2.0 * d.K / h.ndof : 0.0;
        d.step = h.step;
        d.rebuilds = h.rebuilds;
        d.newton_iter_max = h.newton_max;
        d.nlist_max = h.nl_max;
        d.error_index = h.n > 0 ? h.err_id : -1;
        d.error_step = h.n > 0 ? h.err_step : -1;
        d.exact_sum_breaches = h.sum_breaches;
      }
      if (status) status[q] = h.status;
    }
    return MD_OK;
  }
};

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
namespace {

bool use_graphs() {
  const char* e = std::getenv("MD_NO_GRAPH");
  return !(e && e[0] == '1');
}

// Slots and bitmap words one job needs.
int plan_job(const md_params& prm, int kind, const double* surf, int64_t n, const double* x, int64_t* nslots,
             int64_t* nwords) {
  HostJob h;
  h.prm = prm;
  h.surf_kind = kind;
  for (int k = 0; k < MD_SURF_MAXPRM; ++k) h.surf[k] = surf ? surf[k] : 0.0;
  h.n = n;
  Engine::fill_constants(h);
  MDCHK(make_grid(h, x));
  *nslots = Engine::seg_slots(n);
  *nwords = h.bm_words;
  return MD_OK;
}

int check_device(int dev) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) {
    (void)hipGetLastError();
    return MD_EHIP;
  }
  if (dev < 0 || dev >= count) return MD_EINVAL;
  return MD_OK;
}

}  // namespace

struct md_ctx {
  md_params prm{};
  int surf_kind = MD_SURF_NONE;
  double surf[MD_SURF_MAXPRM] = {0};
  bool have_particles = false;
  Engine* eng = nullptr;
  int job = -1;
  bool have_model = false;  // bead model for the next md_set_particles
  ModelDev model{};
  double model_rc = 0.0;    // largest pair cut-off of the model
  std::vector<uint8_t> types;
};

namespace {

// Bead-model tables in the device form: symmetric per type pair, the
// defaults (rc_ab = 0, r0_ab = 0) resolved, the LJ shift at the cut-off.
int build_model(const md_model& m, ModelDev& d, double& rc_max) {
  if (m.ntypes < 1 || m.ntypes > MD_MAX_TYPES || m.beads_per_molecule < 0) return MD_EINVAL;
  static_assert(MD_MAX_TYPES == kMaxTypes, "type table size");
  std::memset(&d, 0, sizeof(d));
  const double c6 = std::pow(2.0, 1.0 / 6.0);
  rc_max = 0.0;
  for (int a = 0; a < m.ntypes; ++a)
    if (!(m.sigma[a] > 0.0) || !std::isfinite(m.sigma[a])) return MD_EINVAL;
  for (int a = 0; a < m.ntypes; ++a)
    for (int b = a; b < m.ntypes; ++b) {
      const double eps = m.eps[a][b], rcin = m.rc[a][b], r0in = m.r0[a][b];
      if (!(eps > 0.0) || !std::isfinite(eps) || !(rcin >= 0.0) || !std::isfinite(rcin) || !(r0in >= 0.0) ||
          !std::isfinite(r0in))
        return MD_EINVAL;
      const double s = 0.5 * (m.sigma[a] + m.sigma[b]);
      const double rc = rcin > 0.0 ? rcin : c6 * s;
      const double sr = s / rc, s6 = sr * sr * sr * sr * sr * sr;
      const double r0 = r0in > 0.0 ? r0in : c6 * (m.sigma[a] + m.sigma[b]) / 4.0;
      for (int q = 0; q < 2; ++q) {
        const int k = q == 0 ? a * kMaxTypes + b : b * kMaxTypes + a;
        d.sig2[k] = s * s;
        d.eps4[k] = 4.0 * eps;
        d.eps24[k] = 24.0 * eps;
        d.rc2[k] = rc * rc;
        d.phic[k] = 4.0 * eps * (s6 * s6 - s6);
        d.r0[k] = r0;
      }
      rc_max = std::max(rc_max, rc);
    }
  if (!(m.kb >= 0.0) || !(m.ka >= 0.0) || !std::isfinite(m.kb) || !std::isfinite(m.ka) ||
      !(m.theta0 >= 0.0 && m.theta0 <= M_PI) || !(m.wall_eps >= 0.0) || !std::isfinite(m.wall_eps) ||
      !std::isfinite(m.wall_radius) || (m.wall_eps > 0.0 && !(m.wall_sigma > 0.0 && std::isfinite(m.wall_sigma))))
    return MD_EINVAL;
  d.kb = m.kb;
  d.ka = m.ka;
  d.theta0 = m.theta0;
  d.wall_eps = m.wall_eps;
  d.wall_sig = m.wall_sigma;
  d.wall_radius = m.wall_radius;
  d.wall_cut = c6 * m.wall_sigma;
  d.ntypes = m.ntypes;
  d.bpm = m.beads_per_molecule;
  return MD_OK;
}

}  // namespace

struct md_pool {
  Engine eng;
};

extern "C" {

const char* md_strerror(int code) {
  switch (code) {
    case MD_OK: return "ok";
    case MD_EINVAL: return "invalid argument";
    case MD_ESTATE: return "call out of order";
    case MD_EOFFSURF: return "particle off the surface or with a normal momentum component";
    case MD_ENEWTON: return "RATTLE Newton iteration did not converge";
    case MD_ENAN: return "non-finite state";
    case MD_ENOMEM: return "out of memory";
    case MD_EAGAIN: return "no room in the pool";
    case MD_EHIP: return "HIP runtime error";
    case MD_ENOTFOUND: return "unknown job";
    default: return "unknown status";
  }
}

int md_create(const md_params* params, md_ctx** out) {
  if (!params || !out) return MD_EINVAL;
  *out = nullptr;
  MDCHK(validate_params(*params));
  MDCHK(check_device(params->device));
  md_ctx* c = new (std::nothrow) md_ctx();
  if (!c) return MD_ENOMEM;
  c->prm = *params;
  *out = c;
  return MD_OK;
}

int md_set_surface(md_ctx* ctx, int kind, const double* prm, int nprm) {
  if (!ctx) return MD_EINVAL;
  const int need = surf_nprm(kind);
  if (need < 0 || nprm < need) return MD_EINVAL;
  MDCHK(validate_surface(kind, prm, ctx->prm));
  ctx->surf_kind = kind;
  for (int k = 0; k < MD_SURF_MAXPRM; ++k) ctx->surf[k] = k < need ? prm[k] : 0.0;
  return MD_OK;
}

int md_set_model(md_ctx* ctx, const md_model* model, const uint8_t* types, int64_t n) {
  if (!ctx) return MD_EINVAL;
  if (!model) {
    ctx->have_model = false;
    ctx->types.clear();
    return MD_OK;
  }
  if (n < 0 || (n > 0 && !types)) return MD_EINVAL;
  if (ctx->prm.pair_kind != MD_PAIR_LJ) return MD_EINVAL;
  ModelDev d;
  double rc_max = 0.0;
  MDCHK(build_model(*model, d, rc_max));
  for (int64_t i = 0; i < n; ++i)
    if (types[i] >= model->ntypes) return MD_EINVAL;
  try {
    ctx->types.assign(types, types + n);
  } catch (...) {
    return MD_ENOMEM;
  }
  ctx->model = d;
  ctx->model_rc = rc_max;
  ctx->have_model = true;
  return MD_OK;
}

int md_set_particles(md_ctx* ctx, int64_t n, const double* x, const double* p, const double* mass,
                     const uint8_t* constrained, const double* fcomb, int64_t step0) {
  if (!ctx || n < 0 || step0 < 0) return MD_EINVAL;
  if (n > 0 && (!x || !p)) return MD_EINVAL;
  md_params prm = ctx->prm;
  if (ctx->have_model) {
    if ((int64_t)ctx->types.size() != n) return MD_EINVAL;
    prm.rc = ctx->model_rc;  // the cell grid and the lists cover the largest pair cut-off
  }
  int64_t nslots = 0, nwords = 0;
  MDCHK(plan_job(prm, ctx->surf_kind, ctx->surf, n, x, &nslots, &nwords));
  {
    // room for the finest grid md_tune may choose (skin 0.2)
    md_params fine = prm;
    fine.skin = 0.2;
    int64_t s2 = 0, w2 = 0;
    if (plan_job(fine, ctx->surf_kind, ctx->surf, n, x, &s2, &w2) == MD_OK) nwords = std::max(nwords, w2);
  }
  Engine* e = ctx->eng;
  if (e && ctx->job >= 0) e->drop(ctx->job);
  ctx->job = -1;
  ctx->have_particles = false;
  if (e && (e->C < nslots || e->BMW < nwords)) {
    delete e;
    e = ctx->eng = nullptr;
  }
  if (!e) {
    e = new (std::nothrow) Engine();
    if (!e) return MD_ENOMEM;
    const int r = e->init(ctx->prm.device, ctx->prm.stream, nslots, nwords, 1);
    if (r != MD_OK) {
      delete e;
      return r;
    }
    ctx->eng = e;
  }
  int j = -1;
  MDCHK(e->admit(prm, ctx->surf_kind, ctx->surf, n, x, p, mass, constrained, fcomb, step0, step0, &j,
                 ctx->have_model ? &ctx->model : nullptr, ctx->have_model ? ctx->types.data() : nullptr));
  ctx->job = j;
  ctx->have_particles = true;
  return MD_OK;
}

int md_step(md_ctx* ctx, int64_t nsteps) {
  if (!ctx || nsteps < 0) return MD_EINVAL;
  if (!ctx->have_particles) return MD_ESTATE;
  Engine* e = ctx->eng;
  HostJob& h = e->jobs[ctx->job];
  if (h.status != MD_OK) return h.status;
  if (nsteps == 0 || h.n == 0) {
    h.step += (h.n == 0) ? nsteps : 0;
    return MD_OK;
  }
  h.target = h.step + nsteps;
  h.done = false;
  e->step_tiles_valid = false;
  const bool graph = use_graphs();
  while (h.step < h.target && h.status == MD_OK) {
    int64_t adv = 0;
    MDCHK(e->run_chunk((int)std::min<int64_t>(h.target - h.step, kMaxChunk), graph, &adv));
  }
  return h.status;
}

int md_get_state(md_ctx* ctx, double* x, double* p, double* fcomb, int64_t* step, md_diag* diag) {
  if (!ctx) return MD_EINVAL;
  if (!ctx->have_particles) return MD_ESTATE;
  Engine* e = ctx->eng;
  if (step) *step = e->jobs[ctx->job].step;
  return e->finish(ctx->job, x, p, fcomb, diag);
}

int md_get_state_dev(md_ctx* ctx, double* x, double* p, double* fcomb, int64_t* step, md_diag* diag) {
  if (!ctx) return MD_EINVAL;
  if (!ctx->have_particles) return MD_ESTATE;
  Engine* e = ctx->eng;
  if (step) *step = e->jobs[ctx->job].step;
  return e->finish(ctx->job, x, p, fcomb, diag, true);
}

int md_get_state_dev_noalloc(md_ctx* ctx, double* x, double* p, double* fcomb, int64_t* step, md_diag* diag) {
  if (!ctx) return MD_EINVAL;
  if (!ctx->have_particles) return MD_ESTATE;
  Engine* e = ctx->eng;
  if (!e->scratch_d) return MD_EHIP;
  HIPCHK(hipSetDevice(ctx->prm.device));
  if (step) *step = e->jobs[ctx->job].step;
  e->no_alloc = true;
  const int rc = e->finish(ctx->job, x, p, fcomb, diag, true, true);
  e->no_alloc = false;
  return rc;
}

int md_set_particles_dev(md_ctx* ctx, int64_t n, const double* x, const double* p, const double* mass,
                         const uint8_t* constrained, const double* fcomb, int64_t step0) {
  if (!ctx || n < 0 || step0 < 0) return MD_EINVAL;
  if (n > 0 && (!x || !p)) return MD_EINVAL;
  if (n == 0) return md_set_particles(ctx, 0, nullptr, nullptr, nullptr, nullptr, nullptr, step0);
  // the inputs are read once, on the context's stream, into host memory: the
  // admission checks (every particle on its surface, momenta tangent) and the
  // cell-grid plan run on the host, as for md_set_particles
  HIPCHK(hipSetDevice(ctx->prm.device));
  hipStream_t s = (hipStream_t)ctx->prm.stream;
  std::vector<double> hx, hp, hm, hf;
  std::vector<uint8_t> hc;
  try {
    hx.resize(3 * n);
    hp.resize(3 * n);
    if (mass) hm.resize(n);
    if (fcomb) hf.resize(3 * n);
    if (constrained) hc.resize(n);
  } catch (...) {
    return MD_ENOMEM;
  }
  HIPCHK(hipMemcpyAsync(hx.data(), x, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hp.data(), p, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s));
  if (mass) HIPCHK(hipMemcpyAsync(hm.data(), mass, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  if (fcomb) HIPCHK(hipMemcpyAsync(hf.data(), fcomb, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s));
  if (constrained) HIPCHK(hipMemcpyAsync(hc.data(), constrained, n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return md_set_particles(ctx, n, hx.data(), hp.data(), mass ? hm.data() : nullptr,
                          constrained ? hc.data() : nullptr, fcomb ? hf.data() : nullptr, step0);
}

int md_tune(md_ctx* ctx, int trial_steps, const double* skins, int nskins, double* best_skin,
            double* best_us_per_step) {
  static const double kDefaultSkins[] = {0.2, 0.3, 0.4, 0.5, 0.6, 0.8};
  if (!ctx || trial_steps <= 0 || nskins < 0 || (nskins > 0 && !skins)) return MD_EINVAL;
  if (!ctx->have_particles) return MD_ESTATE;
  if (!skins || nskins == 0) {
    skins = kDefaultSkins;
    nskins = (int)(sizeof(kDefaultSkins) / sizeof(kDefaultSkins[0]));
  }
  for (int q = 0; q < nskins; ++q)
    if (!(skins[q] > 0.0)) return MD_EINVAL;
  Engine* e = ctx->eng;
  const int j = ctx->job;
  // GPU microseconds per step of one trial: step chunks and list builds (one
  // step first, which takes the list build a new skin forces); step_us: the
  // step chunks alone
  auto trial = [&](double* us, double* step_us) -> int {
    MDCHK(md_step(ctx, 1));
    const md_stats a = e->stats;
    MDCHK(md_step(ctx, trial_steps));
    const md_stats b = e->stats;
    const int64_t steps = b.steps - a.steps;
    const double ks = b.step_kernel_ms - a.step_kernel_ms;
    const double ms = ks + (b.rebuild_ms - a.rebuild_ms);
    *us = steps > 0 ? 1000.0 * ms / (double)steps : 1e300;
    if (step_us) *step_us = steps > 0 ? 1000.0 * ks / (double)steps : 1e300;
    return MD_OK;
  };
  // 1. the step-kernel instance, at the current skin (FP32-class jobs only),
  // by step-kernel time alone (the instance does not change the list builds,
  // whose count per trial would only add noise); each instance is timed twice,
  // in forward and then reverse order, and keeps its faster trial
  const HostJob& h0 = e->jobs[j];
  if (!h0.dev.force_fp64 && !h0.model && h0.n > 0) {
    double v_us[kNumStepVariants];
    for (int v = 0; v < kNumStepVariants; ++v) v_us[v] = 1e300;
    for (int q = 0; q < 2 * kNumStepVariants; ++q) {
      const int v = q < kNumStepVariants ? q : 2 * kNumStepVariants - 1 - q;
      e->set_variant(v);
      double us = 0.0, sus = 0.0;
      MDCHK(trial(&us, &sus));
      v_us[v] = std::min(v_us[v], sus);
    }
    int best_v = 0;
    for (int v = 1; v < kNumStepVariants; ++v)
      if (v_us[v] < v_us[best_v]) best_v = v;
    e->set_variant(best_v);
  }
  // 2. the skin, with that instance
  double best = -1.0, best_us = 1e300;
  for (int q = 0; q < nskins; ++q) {
    if (e->set_skin(j, skins[q]) != MD_OK) continue;
    double us = 0.0;
    MDCHK(trial(&us, nullptr));
    if (us < best_us) {
      best_us = us;
      best = skins[q];
    }
  }
  if (best < 0.0) return MD_ENOMEM;
  MDCHK(e->set_skin(j, best));
  ctx->prm.skin = best;
  if (best_skin) *best_skin = best;
  if (best_us_per_step) *best_us_per_step = best_us;
  return MD_OK;
}

int md_get_stats(md_ctx* ctx, md_stats* stats) {
  if (!ctx || !stats) return MD_EINVAL;
  std::memset(stats, 0, sizeof(*stats));
  if (ctx->eng) {
    *stats = ctx->eng->report();
    if (ctx->have_particles) stats->skin = 2.0 * ctx->eng->jobs[ctx->job].dev.half_skin;
  }
  return MD_OK;
}

void md_destroy(md_ctx* ctx) {
  if (!ctx) return;
  delete ctx->eng;
  delete ctx;
}

size_t md_job_footprint(int64_t n, int surface_kind, const double* surface_prm, const md_params* params) {
  if (!params || n < 0) return 0;
  // the grid of a surface-less job depends on the particles; size it as a cube
  // holding them at unit density
  int64_t nslots = 0, nwords = 0;
  if (surface_kind == MD_SURF_NONE) {
    nslots = Engine::seg_slots(n);
    nwords = n / 8 + 64;
  } else if (plan_job(*params, surface_kind, surface_prm, n, nullptr, &nslots, &nwords) != MD_OK) {
    return 0;
  }
  return (size_t)((double)nslots * slot_bytes(kDefaultKmax + kDefaultKmax / 2, kDefaultHcap)) + (size_t)nwords * 8;
}

int md_pool_create(size_t hbm_budget_bytes, int max_jobs, int device, void* stream, md_pool** out) {
  if (!out || max_jobs <= 0 || hbm_budget_bytes < (1u << 20)) return MD_EINVAL;
  *out = nullptr;
  MDCHK(check_device(device));
  md_pool* pl = new (std::nothrow) md_pool();
  if (!pl) return MD_ENOMEM;
  const double per_slot = slot_bytes(kDefaultKmax + kDefaultKmax / 2, kDefaultHcap);
  const int64_t slots = (int64_t)(0.75 * (double)hbm_budget_bytes / per_slot);
  const int64_t words = (int64_t)(0.25 * (double)hbm_budget_bytes / 8.0);
  const int r = pl->eng.init(device, stream, slots, words, max_jobs);
  if (r != MD_OK) {
    delete pl;
    return r;
  }
  *out = pl;
  return MD_OK;
}

int md_pool_admit(md_pool* pool, const md_job_desc* job, int* job_id) {
  if (!pool || !job || !job_id) return MD_EINVAL;
  if (job->nsteps < 0 || job->step0 < 0) return MD_EINVAL;
  MDCHK(validate_surface(job->surface_kind, job->surface_prm, job->params));
  md_params prm = job->params;
  ModelDev md;
  if (job->model) {
    double rc_max = 0.0;
    MDCHK(build_model(*job->model, md, rc_max));
    if (job->n > 0 && !job->types) return MD_EINVAL;
    for (int64_t i = 0; i < job->n; ++i)
      if (job->types[i] >= job->model->ntypes) return MD_EINVAL;
    prm.rc = rc_max;  // the cell grid and the lists cover the largest pair cut-off
  }
  return pool->eng.admit(prm, job->surface_kind, job->surface_prm, job->n, job->x, job->p, job->mass,
                         job->constrained, nullptr, job->step0, job->step0 + job->nsteps, job_id,
                         job->model ? &md : nullptr, job->model ? job->types : nullptr);
}

int md_pool_run(md_pool* pool, int steps_chunk) {
  if (!pool || steps_chunk < 0) return MD_EINVAL;
  Engine& e = pool->eng;
  MDCHK(e.drain());
  const bool graph = use_graphs();
  int64_t left = steps_chunk;
  while (left > 0) {
    int64_t adv = 0;
    MDCHK(e.run_chunk((int)std::min<int64_t>(left, kPoolChunk), graph, &adv, true));
    if (adv <= 0) {
      bool any = false;
      for (int j = 0; j < e.max_jobs; ++j) any = any || e.steppable(e.jobs[j]);
      if (!any) break;
      continue;
    }
    left -= adv;
  }
  return MD_OK;
}

int md_pool_launch(md_pool* pool, int steps_chunk) {
  if (!pool || steps_chunk < 0) return MD_EINVAL;
  Engine& e = pool->eng;
  MDCHK(e.drain());
  if (steps_chunk == 0) return MD_OK;
  return e.enqueue_chunk((int)std::min<int64_t>(steps_chunk, kPoolChunk), use_graphs(), true);
}

int md_pool_poll(md_pool* pool, int* done_ids, int cap, int* ndone) {
  if (!pool || !ndone || (cap > 0 && !done_ids)) return MD_EINVAL;
  Engine& e = pool->eng;
  MDCHK(e.drain());
  int c = 0;
  for (int j = 0; j < e.max_jobs && c < cap; ++j) {
    HostJob& h = e.jobs[j];
    if (!h.used || h.reported) continue;
    if (h.done || h.status != MD_OK || h.step >= h.target) {
      h.reported = true;
      done_ids[c++] = j;
    }
  }
  *ndone = c;
  return MD_OK;
}

int md_pool_fetch(md_pool* pool, int job_id, double* x, double* p, md_diag* diag) {
  if (!pool || job_id < 0 || job_id >= pool->eng.max_jobs) return MD_ENOTFOUND;
  if (!pool->eng.jobs[job_id].used) return MD_ENOTFOUND;
  MDCHK(pool->eng.drain());
  return pool->eng.finish(job_id, x, p, nullptr, diag);
}

int md_pool_fetch_many(md_pool* pool, const int* job_ids, int n, double* const* x, double* const* p, md_diag* diag,
                       int* status) {
  if (!pool || n < 0 || (n > 0 && !job_ids)) return MD_EINVAL;
  if (n == 0) return MD_OK;
  MDCHK(pool->eng.drain());
  return pool->eng.finish_many(job_ids, n, x, p, diag, status);
}

int md_pool_release(md_pool* pool, int job_id) {
  if (!pool || job_id < 0 || job_id >= pool->eng.max_jobs) return MD_ENOTFOUND;
  if (!pool->eng.jobs[job_id].used) return MD_ENOTFOUND;
  MDCHK(pool->eng.drain());
  pool->eng.drop(job_id);
  return MD_OK;
}

int md_pool_usage(md_pool* pool, int* jobs, int64_t* particles, size_t* bytes) {
  if (!pool) return MD_EINVAL;
  int nj = 0;
  int64_t np = 0, slots = 0, words = 0;
  for (const HostJob& h : pool->eng.jobs)
    if (h.used) {
      ++nj;
      np += h.n;
      slots += h.seg;
      words += h.bm_words;
    }
  if (jobs) *jobs = nj;
  if (particles) *particles = np;
  if (bytes) *bytes = (size_t)((double)slots * slot_bytes(pool->eng.kmax, pool->eng.hcap)) + (size_t)words * 8;
  return MD_OK;
}

int md_pool_get_stats(md_pool* pool, md_stats* stats) {
  if (!pool || !stats) return MD_EINVAL;
  *stats = pool->eng.report();
  return MD_OK;
}

void md_pool_destroy(md_pool* pool) {
  if (!pool) return;
  (void)pool->eng.drain();
  delete pool;
}

}  // extern "C"
