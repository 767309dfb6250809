// kernels.hpp -- the list build, sort, diagnostics and bookkeeping kernels of
// the RATTLE + Langevin hot path (gfx950); the step kernels are in step.hpp.
#pragma once

#include "step.hpp"

namespace mdk {

// ---------------------------------------------------------------------------
// Neighbour-list build: occupied-cell bitmap -> compact cell index by popcount
// prefix -> counting sort of particles into raster cell order -> lists.
// ---------------------------------------------------------------------------

// Cell coordinate along dimension k: wrapped into the grid when periodic (in
// FP64, exact for the integers involved; no 64-bit integer division), clamped
// to the edge cells otherwise.  The final clamp also keeps a wrap rounded far
// from the box, or a NaN, inside the grid.
__device__ __forceinline__ int cell_coord(const JobDev& J, int k, double v) {
  double c = floor((v - J.glo[k]) * J.inv_cs[k]);
  const double nc = (double)J.nc[k];
  if (J.periodic[k]) c -= nc * floor(c / nc);
  return (int)fmin(fmax(c, 0.0), nc - 1.0);
}

__device__ __forceinline__ uint32_t raster_of(const JobDev& J, int cx, int cy, int cz) {
  return ((uint32_t)cx * (uint32_t)J.nc[1] + (uint32_t)cy) * (uint32_t)J.nc[2] + (uint32_t)cz;
}

// Zero [base + start, base + start + len) for each range.
struct Range {
  int64_t start;
  int64_t len;
};

// Clears words [start, start + len) of each range: ranges 0 .. n0-1 of array
// a0, the next n1 of a1, the rest of a2 (one launch for all three; range
// q0 + blockIdx.y per row of workgroups).
__global__ void k_zero_ranges(uint32_t* __restrict__ a0, uint32_t* __restrict__ a1, uint32_t* __restrict__ a2,
                              const Range* __restrict__ ranges, int n0, int n1, int q0) {
  const int q = q0 + (int)blockIdx.y;
  const Range r = ranges[q];
  uint32_t* __restrict__ base = q < n0 ? a0 : (q < n0 + n1 ? a1 : a2);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < r.len; k += (int64_t)gridDim.x * blockDim.x)
    base[r.start + k] = 0u;
}

// Wavefront-level combining of atomics on equal addresses.  After a build the
// particles are stored in cell order, so neighbouring lanes usually share a
// bitmap word / cell counter.  Lanes are grouped into runs of equal keys; the
// runs of a wavefront issue their atomics in one instruction (runs with equal
// keys that are not adjacent simply issue separate atomics).
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

__device__ __forceinline__ unsigned long long lanemask_le(int lane) {
  return lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
}

// First lane of the run of equal keys that contains this lane.
__device__ __forceinline__ int run_start(uint32_t key, int lane, unsigned long long* heads_out) {
  const uint32_t prev = __shfl_up(key, 1, 64);
  const bool head = lane == 0 || prev != key;
  const unsigned long long heads = __ballot(head);
  *heads_out = heads;
  return 63 - __clzll((long long)(heads & lanemask_le(lane)));
}

__global__ void __launch_bounds__(kTile) k_mark(DevBufs B, const int* __restrict__ tile_job,
                                                const int64_t* __restrict__ tile_first) {
  const int job = uniform_int(tile_job[blockIdx.x]);
  const JobDev& J = B.jobs[job];
  const int64_t i = uniform_i64(tile_first[blockIdx.x]) + threadIdx.x;
  const bool valid = i < J.off + J.n;
  uint32_t key = kNoKey, bits = 0u;
  if (valid) {
    const double* X = B.X[J.xcur];
    const double px = X[3 * i], py = X[3 * i + 1], pz = X[3 * i + 2];
    const int cx = cell_coord(J, 0, px), cy = cell_coord(J, 1, py), cz = cell_coord(J, 2, pz);
    const uint32_t r = raster_of(J, cx, cy, cz);
    B.RASTER[i] = r;
    key = r >> 5;
    bits = 1u << (r & 31);
  }
  const int lane = threadIdx.x & 63;
  unsigned long long heads;
  const int start = run_start(key, lane, &heads);
  // OR over the run, accumulated towards its last lane
  uint32_t v = bits;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, o, 64);
    if (lane - o >= start) v |= t;
  }
  const bool tail = lane == 63 || ((heads >> (lane + 1)) & 1ull);
  if (tail && key != kNoKey) atomicOr(&B.BM[J.bm_off + key], v);
  // a list build starts the job's bookkeeping afresh (stored last, so that no
  // read of the job record has to wait behind it)
  if (i == J.off) B.book[job] = fresh_book();
}

__global__ void __launch_bounds__(kTile) k_count(DevBufs B, const int* __restrict__ tile_job,
                                                 const int64_t* __restrict__ tile_first) {
  const int job = uniform_int(tile_job[blockIdx.x]);
  const JobDev& J = B.jobs[job];
  const int64_t i = uniform_i64(tile_first[blockIdx.x]) + threadIdx.x;
  const bool valid = i < J.off + J.n;
  uint32_t key = kNoKey;
  if (valid) {
    const uint32_t r = B.RASTER[i];
    const int64_t w = J.bm_off + (r >> 5);
    key = B.WOFF[w] + __popc(B.BM[w] & ((1u << (r & 31)) - 1u));
    B.CID[i] = key;
  }
  const int lane = threadIdx.x & 63;
  unsigned long long heads;
  const int start = run_start(key, lane, &heads);
  uint32_t base = 0u;
  if (start == lane && key != kNoKey) {
    const unsigned long long later = heads & ~lanemask_le(lane);
    const int next = later ? __ffsll((long long)later) - 1 : 64;
    base = atomicAdd(&B.CCNT[J.off + key], (uint32_t)(next - lane));
  }
  base = __shfl(base, start, 64);
  if (valid) B.RANK[i] = base + (uint32_t)(lane - start);
}

// Move every slot's state to its place in the new (cell) order: slot i goes
// to d = the start of its cell + its rank in the cell.  Consecutive threads
// read consecutive slots (whole cache lines); the writes follow the
// permutation, which moves most slots only a few places since the last sort,
// so they land in the same cache lines.  Jobs with a bead model also get the
// inverse permutation by particle index (the bonded terms find the beads of a
// molecule through it).  The noise cache (the last step's normals) moves with
// the momenta.
__global__ void __launch_bounds__(kTile) k_move(DevBufs B, const int* __restrict__ tile_job,
                                                const int64_t* __restrict__ tile_first) {
  const int job = uniform_int(tile_job[blockIdx.x]);
  const JobDev& J = B.jobs[job];
  const int64_t i = uniform_i64(tile_first[blockIdx.x]) + threadIdx.x;
  const int64_t off = J.off;
  if (i >= off + J.n) return;
  const double* __restrict__ Xs = B.X[J.xcur];
  double* __restrict__ Xd = B.X[J.xcur ^ 1];
  const double* __restrict__ Ps = B.P[J.pcur];
  double* __restrict__ Pd = B.P[J.pcur ^ 1];
  // every load before the first store: source and destination are different
  // buffers, and this way the loads are in flight together
  const uint32_t cid = B.CID[i], rank = B.RANK[i];
  double x[3], p[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    x[k] = Xs[3 * i + k];
    p[k] = Ps[3 * i + k];
  }
  const int sc = J.scur;
  const bool per_mass = !J.uniform_mass, model = J.model != 0, f64 = J.force_fp64 != 0;
  const uint32_t id = B.ID[sc][i];
  const uint8_t flag = B.FLG[sc][i];
  const double mass = per_mass ? B.MASS[sc][i] : 0.0;
  const uint8_t type = model ? B.TYPE[sc][i] : (uint8_t)0;
  double nz[3];
  if (f64) {
    const double* zs = B.NZD[J.pcur];
#pragma unroll
    for (int k = 0; k < 3; ++k) nz[k] = zs[3 * i + k];
  } else {
    const float* zs = B.NZF[J.pcur];
#pragma unroll
    for (int k = 0; k < 3; ++k) nz[k] = (double)zs[3 * i + k];
  }
  const int64_t d = off + B.CSTART[off + cid] + rank;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Xd[3 * d + k] = x[k];
    Pd[3 * d + k] = p[k];
  }
  if (f64) {
    double* zd = B.NZD[J.pcur ^ 1];
#pragma unroll
    for (int k = 0; k < 3; ++k) zd[3 * d + k] = nz[k];
  } else {
    float* zd = B.NZF[J.pcur ^ 1];
#pragma unroll
    for (int k = 0; k < 3; ++k) zd[3 * d + k] = (float)nz[k];
  }
  B.ID[sc ^ 1][d] = id;
  B.FLG[sc ^ 1][d] = flag;
  if (per_mass) B.MASS[sc ^ 1][d] = mass;
  uint32_t w = id;
  if (model) {
    // bead model: the type rides in the top two bits of the record's index
    B.TYPE[sc ^ 1][d] = type;
    w |= (uint32_t)type << kTypeShift;
    B.INV[off + id] = (uint32_t)(d - off);
  }
  B.PK[d] = make_float4((float)x[0], (float)x[1], (float)x[2], __uint_as_float(w));
}

// Occupied cells with raster index below r, for the compact cell index.
__device__ __forceinline__ uint32_t cells_before(const DevBufs& B, const JobDev& J, uint32_t r) {
  const int64_t w = J.bm_off + (r >> 5);
  return B.WOFF[w] + __popc(B.BM[w] & ((1u << (r & 31)) - 1u));
}

// Cell coordinate c + d along dimension k for a stencil offset d in {-1,0,1}:
// wrapped when periodic (offsets that would repeat a cell when the periodic
// count is below 3 are dropped), dropped outside a non-periodic grid.
__device__ __forceinline__ bool stencil_coord(const JobDev& J, int k, int c, int d, int& out) {
  const int nc = J.nc[k];
  if (J.periodic[k]) {
    if (nc < 3 && (d < 0 || d >= nc)) return false;
    const int v = c + d;
    out = v < 0 ? v + nc : (v >= nc ? v - nc : v);
    return true;
  }
  out = c + d;
  return out >= 0 && out < nc;
}

// z cells of the stencil around cz: [za0, zb0] and, when z wraps, [za1, zb1].
__device__ __forceinline__ void z_runs(const JobDev& J, int cz, int& za0, int& zb0, int& za1, int& zb1) {
  const int ncz = J.nc[2];
  za1 = 0, zb1 = -1;
  if (J.periodic[2] && ncz >= 3) {
    if (cz == 0) {
      za0 = 0, zb0 = 1, za1 = ncz - 1, zb1 = ncz - 1;
    } else if (cz == ncz - 1) {
      za0 = 0, zb0 = 0, za1 = cz - 1, zb1 = cz;
    } else {
      za0 = cz - 1, zb0 = cz + 1;
    }
  } else if (J.periodic[2]) {
    za0 = 0, zb0 = ncz - 1;
  } else {
    za0 = cz > 0 ? cz - 1 : 0;
    zb0 = cz + 1 < ncz ? cz + 1 : ncz - 1;
  }
}

// Key of stencil column col (0..8) of cell column (cx, cy): x nc_y + y, or
// kNoCol off a non-periodic grid.
__device__ __forceinline__ uint32_t column_key(const JobDev& J, int cx, int cy, int col) {
  int ax = 0, ay = 0;
  const bool ok = stencil_coord(J, 0, cx, col / 3 - 1, ax) & stencil_coord(J, 1, cy, col % 3 - 1, ay);
  return ok ? (uint32_t)ax * (uint32_t)J.nc[1] + (uint32_t)ay : 0xFFFFFFFFu;
}

// Slot runs [rb, re) (relative to the job) of cells z in [za, zb] of stencil
// columns C0 .. C1-1 of (cx, cy), looked up together in two rounds of loads:
// per column the bitmap word of its first cell, the word after it when the
// run's end falls there (za..zb spans at most three cells, so the end is in
// one of the two), and the first word's popcount prefix; then the two cell
// starts.  An off-grid column gives an empty run.
template <int C0, int C1>
__device__ __forceinline__ void column_runs(const DevBufs& B, const JobDev& J, int cx, int cy, int za, int zb,
                                            uint32_t* rb, uint32_t* re) {
  constexpr int G = C1 - C0;
  const uint32_t ncy = (uint32_t)J.nc[1], ncz = (uint32_t)J.nc[2];
  // the job's bitmap, popcount prefix and cell starts (uniform bases, 32-bit
  // per-lane offsets)
  const uint32_t* __restrict__ bm = B.BM + J.bm_off;
  const uint32_t* __restrict__ woff = B.WOFF + J.bm_off;
  const uint32_t* __restrict__ cstart = B.CSTART + J.off;
  const uint32_t dz = (uint32_t)(zb - za + 1);  // cells in the run (at most three)
  uint32_t ra[G], bm0[G], bm1[G], wo[G];
  uint32_t okm = 0u;  // bit u: column C0 + u is on the grid
#pragma unroll
  for (int u = 0; u < G; ++u) {
    const int col = C0 + u;
    int ax = 0, ay = 0;
    const bool ok = stencil_coord(J, 0, cx, col / 3 - 1, ax) & stencil_coord(J, 1, cy, col % 3 - 1, ay);
    if (!ok) ax = 0, ay = 0;  // looks up column (0, 0), dropped below
    okm |= ok ? 1u << u : 0u;
    ra[u] = ((uint32_t)ax * ncy + (uint32_t)ay) * ncz + (uint32_t)za;
    const uint32_t wa = ra[u] >> 5;
    bm0[u] = bm[wa];
    wo[u] = woff[wa];
    // the end's word, when it is the next one (always inside the job's words:
    // the end of the last z-run is addressable)
    bm1[u] = ((ra[u] + dz) >> 5) != wa ? bm[wa + 1u] : 0u;
  }
#pragma unroll
  for (int u = 0; u < G; ++u) {
    const uint32_t rz = ra[u] + dz;
    const uint32_t ia = wo[u] + __popc(bm0[u] & ((1u << (ra[u] & 31)) - 1u));
    const uint32_t mz = (1u << (rz & 31)) - 1u;
    const uint32_t iz = (rz >> 5) != (ra[u] >> 5) ? wo[u] + __popc(bm0[u]) + __popc(bm1[u] & mz)
                                                  : wo[u] + __popc(bm0[u] & mz);
    rb[C0 + u] = cstart[ia];
    re[C0 + u] = cstart[iz];
  }
#pragma unroll
  for (int u = 0; u < G; ++u)
    if (!((okm >> u) & 1u)) re[C0 + u] = rb[C0 + u];
}

// The runs of all 9 stencil columns, in two groups of lookups.
__device__ __forceinline__ void column_runs9(const DevBufs& B, const JobDev& J, int cx, int cy, int za, int zb,
                                             uint32_t* rb, uint32_t* re) {
  column_runs<0, 5>(B, J, cx, cy, za, zb, rb, re);
  column_runs<5, 9>(B, J, cx, cy, za, zb, rb, re);
}

// Exclusive scan over the 256 threads of a workgroup (every thread calls it);
// *total receives the sum.  sh: 4 words of LDS.
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
  const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  uint32_t before = 0u, tot = 0u;
#pragma unroll
  for (int q = 0; q < kNlistBlock / 64; ++q) {
    const uint32_t s = sh[q];
    if (q < w) before += s;
    tot += s;
  }
  total = tot;
  __syncthreads();
  return before + x - v;
}

// Neighbour-list build.  One workgroup per tile (256 slots of the freshly
// sorted raster cell order), one lane per slot:
//  0. each lane looks up the slot runs of its 9 stencil columns (cells z-1..z+1
//     of each; three columns' lookups in flight together) and keeps them in
//     registers;
//  1. the first lane of each cell (the tile's lanes of one cell are
//     consecutive) puts, per column, the hull of the slots the cell needs
//     into an LDS table of the tile's columns; the hulls, one after another,
//     number the tile's candidates;
//  2. each lane walks its 9 runs over the packed FP32 candidate records, four
//     at a time with the next four loading, and appends the candidate numbers
//     of those inside the list radius without branching (a rejected candidate
//     is overwritten by the next one); its own slot is found like any other;
//  3. kept candidates in the tile become local indices (the lane's own slot
//     leaves the list), the others are marked in a bitmap over candidate
//     numbers; the halo is the marked candidates in candidate order; list
//     entries become window indices (own slots 0..255, halo 256 + rank) and
//     are written as 16-bit entries, with the halo list of the tile.
// FP64 class: lists sorted by particle index (the order of the FP64 sums).
// FP32 class: lists in the order found.
// FP64-class and bead-model jobs look up the index (and type) of each window
// entry in a table of the window's record words, made with the halo list.
// Bead model: each bead's bonded partners (beads id-2 .. id+2 of its
// molecule, found through the inverse permutation) join the halo like list
// entries, and their window entries are stored in BW for the step kernel.
// The FP32 distance test uses the list radius widened by a bound on the FP32
// rounding of both positions and of the separation (times eight), so it
// accepts every pair closer than the list radius; the few extra pairs it may
// accept lie beyond the cut-off and add nothing to the forces.
constexpr int kColCap = 256;     // distinct stencil columns of one tile
constexpr int kCandCap = 16384;  // candidates of one tile
constexpr uint32_t kNoCol = 0xFFFFFFFFu;
constexpr int kNlistRows = 2;    // list rows in LDS beyond kmax

// FP32 minimum image with box lengths L and inverses iL (both 0 along a
// non-periodic axis, where the correction vanishes).
__device__ __forceinline__ void min_image_f(const float* L, const float* iL, float& dx, float& dy, float& dz) {
  dx = fmaf(-L[0], rintf(dx * iL[0]), dx);
  dy = fmaf(-L[1], rintf(dy * iL[1]), dy);
  dz = fmaf(-L[2], rintf(dz * iL[2]), dz);
}

// One row of a list (entries k .. k+7 of slot i).  Streaming (as the step's
// state stores, when the data exceed the Infinity Cache): the lists are read
// in the next step, not in this launch.
template <bool kStream>
__device__ __forceinline__ void store_row(uint16_t* NL, int64_t C, int k, int64_t i, const uint32_t* e) {
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const v4u row = {e[0] | (e[1] << 16), e[2] | (e[3] << 16), e[4] | (e[5] << 16), e[6] | (e[7] << 16)};
  v4u* dst = reinterpret_cast<v4u*>(NL) + (int64_t)(k / kRow) * C + i;
  if (kStream)
    __builtin_nontemporal_store(row, dst);
  else
    *dst = row;
}

// The table entry of column key (read only), or -1.
__device__ __forceinline__ int column_slot(const uint32_t* ckey, uint32_t key) {
  uint32_t h = (key * 0x9E3779B1u) >> 24;
  for (int probe = 0; probe < kColCap; ++probe) {
    const uint32_t k = ckey[h];
    if (k == key) return (int)h;
    if (k == kNoCol) return -1;
    h = (h + 1u) & (kColCap - 1);
  }
  return -1;
}

// kWide: the instance for builds that include FP64-class or bead-model jobs
// (typed radii, the window-record table, the ordering by particle index).
// The FP32-class instance is held to 80 registers (6 wavefronts per SIMD);
// the wide one keeps the compiler's allocation.
// jobs, models: B.jobs and B.models as no-alias arguments (scalar loads).
template <bool kWide, bool kStream>
__global__ void __launch_bounds__(kNlistBlock) __attribute__((amdgpu_waves_per_eu(kWide ? 1 : 6, 8)))
k_nlist(DevBufs B, const JobDev* __restrict__ jobs, const ModelDev* __restrict__ models,
        const int* __restrict__ tile_job, const int64_t* __restrict__ tile_first) {
  // codes of kept neighbours: own-tile slots as kOwn | local index, others as
  // their candidate number
  using code_t = uint16_t;
  constexpr uint32_t kOwn = 0x8000u;
  // codes [kmax + kNlistRows][256] (kmax + 1 entries with the lane's own slot, then
  // a row for the appends beyond the capacity);
  // wide instance: then the record words (particle index, bead type) of the
  // window, [256 + hcap] (in global memory, B.KKEY, when they would not fit)
  extern __shared__ uint32_t dyn[];
  __shared__ uint32_t ckey[kColCap], cb[kColCap], ce[kColCap], coff[kColCap];
  __shared__ uint32_t bits[kCandCap / 32], wpre[kCandCap / 32];
  __shared__ uint32_t scan_sh[kNlistBlock / 64];
  __shared__ uint32_t span_lo, span_hi, nhull;
  __shared__ int fail;
  const int kmax = B.kmax;
  code_t* kid = reinterpret_cast<code_t*>(dyn);
  const uint32_t wlen = (uint32_t)kTile + (uint32_t)B.hcap;  // window length
  uint32_t* wrec = B.KKEY ? B.KKEY + (size_t)blockIdx.x * wlen : dyn + (size_t)(kmax + kNlistRows) * kNlistBlock / 2;
  const int tile = (int)blockIdx.x;
  const int job = uniform_int(tile_job[tile]);
  const JobDev& J = jobs[job];
  JobBook& K = B.book[job];
  const int lane = (int)threadIdx.x;
  const int wl = lane & 63;
  const int64_t first = uniform_i64(tile_first[tile]);
  const int64_t i = first + lane;
  const int64_t base = J.off;
  const uint32_t first_local = (uint32_t)(first - base);
  const int64_t gt = first / kTile;
  const bool valid = i < J.off + J.n;
  const int64_t C = B.C;
  if (J.pair_kind == kPairNone) {
    // no pair potential: empty lists (the build only sorts)
    if (valid) B.NCNT[i] = 0u;
    if (lane == 0) B.HCNT[gt] = 0u;
    if (lane % kGroup == 0 && valid) {
      B.NLSTAT[2 * (i / kGroup)] = 0u;
      B.NLSTAT[2 * (i / kGroup) + 1] = 0u;
    }
    return;
  }
  const bool sorted = kWide && J.force_fp64;
  const bool typed = kWide && J.model;
  ckey[lane] = kNoCol;
  cb[lane] = 0xFFFFFFFFu;
  ce[lane] = 0u;
  for (int w = lane; w < kCandCap / 32; w += kNlistBlock) bits[w] = 0u;
  if (lane == 0) fail = 0, span_lo = 0xFFFFFFFFu, span_hi = 0u;
  const double* __restrict__ X = B.X[J.xcur ^ 1];  // the sorted copies written by k_move
  const float4* __restrict__ PK = B.PK + base;
  if (kWide) wrec[lane] = valid ? __float_as_uint(PK[first_local + lane].w) : 0u;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  int cx = 0, cy = 0, cz = 0;
  if (valid) {
    xi = X[3 * i];
    yi = X[3 * i + 1];
    zi = X[3 * i + 2];
    cx = cell_coord(J, 0, xi);
    cy = cell_coord(J, 1, yi);
    cz = cell_coord(J, 2, zi);
  }
  int za0, zb0, za1, zb1;
  z_runs(J, cz, za0, zb0, za1, zb1);
  __syncthreads();
  // the lane's 9 stencil columns: run 0 (z in [za0, zb0]) of each; when z
  // wraps there is a second run (z in [za1, zb1]), looked up where needed
  const bool wrap = valid && zb1 >= za1;
  uint32_t rb[9], re[9];
  column_runs9(B, J, cx, cy, za0, zb0, rb, re);
  // 1. the tile's columns: the first lane of each cell finds the hulls of the
  // runs its cell needs per column, and their span over the whole tile
  const uint32_t rkey = valid ? raster_of(J, cx, cy, cz) : kNoKey;
  unsigned long long heads;
  const int rs = run_start(rkey, wl, &heads);  // every lane takes part (shuffle, ballot)
  const bool head = valid && rs == wl;
  uint32_t lo[9], hi[9];
#pragma unroll
  for (int col = 0; col < 9; ++col) lo[col] = rb[col], hi[col] = re[col];
  if (head) {
    if (wrap) {
      uint32_t b1[9], e1[9];
      column_runs9(B, J, cx, cy, za1, zb1, b1, e1);
#pragma unroll
      for (int col = 0; col < 9; ++col) {
        if (e1[col] <= b1[col]) continue;
        if (hi[col] <= lo[col])
          lo[col] = b1[col], hi[col] = e1[col];
        else
          lo[col] = min(lo[col], b1[col]), hi[col] = max(hi[col], e1[col]);
      }
    }
    uint32_t smin = 0xFFFFFFFFu, smax = 0u;
#pragma unroll
    for (int col = 0; col < 9; ++col)
      if (hi[col] > lo[col]) smin = min(smin, lo[col]), smax = max(smax, hi[col]);
    atomicMin(&span_lo, smin);
    atomicMax(&span_hi, smax);
  }
  __syncthreads();
  // Candidate numbers: the slot's offset in the span of all the tile's runs
  // when that span fits the bitmap (always for jobs of at most kCandCap
  // particles, among them sparse tiles whose stencils cover many columns),
  // else by columns: the hulls of the tile's distinct stencil columns, one
  // after another (large dense jobs, whose tiles cover few columns but whose
  // span reaches over several rows of cells)
  const uint32_t span = span_hi > span_lo ? span_hi - span_lo : 0u;
  const bool by_span = span <= (uint32_t)kCandCap;
  if (!by_span && head) {
#pragma unroll
    for (int col = 0; col < 9; ++col) {
      if (hi[col] <= lo[col]) continue;
      const uint32_t key = column_key(J, cx, cy, col);
      uint32_t h = (key * 0x9E3779B1u) >> 24;
      int found = -1;
      for (int probe = 0; probe < kColCap; ++probe) {
        const uint32_t old = atomicCAS(&ckey[h], kNoCol, key);
        if (old == kNoCol || old == key) {
          found = (int)h;
          break;
        }
        h = (h + 1u) & (kColCap - 1);
      }
      if (found < 0) {
        fail = 1;
        break;
      }
      atomicMin(&cb[found], lo[col]);
      atomicMax(&ce[found], hi[col]);
    }
  }
  __syncthreads();
  // candidate numbering by columns: the hulls (disjoint slot ranges) one after
  // another in slot order, so that numbers grow with the slot as in the span
  // numbering and the tile's own slots have consecutive numbers.  coff: per
  // table entry, number minus slot in its hull; then, in slot order, the
  // hulls' first numbers (scoff, in place of cb) and first slots (scb, in
  // place of ce), the occupied entries listed in wpre meanwhile
  uint32_t M = span;
  if (!by_span) {
    const bool occ = ckey[lane] != kNoCol;
    const uint32_t my = cb[lane], len = occ ? ce[lane] - my : 0u;
    uint32_t nh = 0u;
    block_scan(len, scan_sh, M);
    const uint32_t r = block_scan(occ ? 1u : 0u, scan_sh, nh);
    uint32_t* hidx = wpre;
    if (occ) hidx[r] = (uint32_t)lane;
    __syncthreads();
    uint32_t off = 0u, rank = 0u;
    if (occ) {
      for (uint32_t q = 0; q < nh; ++q) {
        const uint32_t j = hidx[q], bj = cb[j];
        if (bj < my) off += ce[j] - bj, ++rank;
      }
    }
    __syncthreads();
    uint32_t *scoff = cb, *scb = ce;
    coff[lane] = off - my;
    if (occ) scoff[rank] = off, scb[rank] = my;
    if (lane == 0) nhull = nh;
    M = M > (uint32_t)kCandCap || fail ? 0xFFFFFFFFu : M;
  }
  __syncthreads();
  if (M > (uint32_t)kCandCap) {
    // neither numbering fits: the job stops with an error
    if (lane == 0) {
      atomicOr(&K.build_fail, 1);
      atomicMin(&K.stop_at, (long long)J.step0);
      B.HCNT[gt] = 0u;
    }
    if (valid) B.NCNT[i] = 0u;
    if (lane % kGroup == 0 && valid) {
      B.NLSTAT[2 * (i / kGroup)] = 0u;
      B.NLSTAT[2 * (i / kGroup) + 1] = 0u;
    }
    return;
  }
  // 2. this lane's stencil walk
  int cnt = 0;
  // the lane's particle index and its molecule [mstart, mstart + bpm) (bpm = 0:
  // no molecules)
  const uint32_t myid = kWide && valid ? B.ID[J.scur ^ 1][i] : 0u;
  const uint32_t bpm = (uint32_t)J.bpm, mstart = bpm != 0u ? (myid / bpm) * bpm : 0u;
  if (valid) {
    const bool anyper = uniform_int(J.periodic[0] | J.periodic[1] | J.periodic[2]) != 0;
    double lper = 0.0;
    float pL[3], piL[3];
    for (int k = 0; k < 3; ++k) {
      if (J.periodic[k]) lper = fmax(lper, J.box_len[k]);
      pL[k] = J.periodic[k] ? (float)J.box_len[k] : 0.0f;
      piL[k] = J.periodic[k] ? (float)J.inv_box_len[k] : 0.0f;
    }
    const double rl = sqrt(J.rlist2);
    const double delta = 0x1p-21 * (2.0 * fmax(fabs(xi), fmax(fabs(yi), fabs(zi))) + 3.0 * rl + lper);
    const float thr = (float)((rl + delta) * (rl + delta) * (1.0 + 0x1p-20));
    const float xf = (float)xi, yf = (float)yi, zf = (float)zi;
    // bead model: list radius per partner type, rc_ab + skin (the rounding
    // bound above covers the shorter radii too); partners of the same
    // molecule are left out
    float tthr[kMaxTypes];
    if (kWide) {
      const int ti = typed ? (int)B.TYPE[J.scur ^ 1][i] : 0;
      const double skin = 2.0 * J.half_skin;
      const ModelDev& Mo = models[job];
#pragma unroll
      for (int b = 0; b < kMaxTypes; ++b) {
        const double r = typed ? sqrt(Mo.rc2[ti * kMaxTypes + b]) + skin : rl;
        tthr[b] = (float)((r + delta) * (r + delta) * (1.0 + 0x1p-20));
      }
    }
    // four candidates r[0..3] numbered t .. t+3 (rem: candidates left from t);
    // every one is written at the next free row, a kept one advances it (row
    // kmax + 1 takes what does not fit)
    auto test4 = [&](const float4* r, int rem, uint32_t t) {
      const int row0 = min(cnt, kmax + 1);
      int tk = 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        float dx = xf - r[u].x, dy = yf - r[u].y, dz = zf - r[u].z;
        if (anyper) min_image_f(pL, piL, dx, dy, dz);
        const float d2 = dx * dx + dy * dy + dz * dz;
        const uint32_t w = __float_as_uint(r[u].w);
        bool take;
        if (kWide) {
          const uint32_t tj = w >> kTypeShift;
          const float tt = tj == 0u ? tthr[0] : (tj == 1u ? tthr[1] : (tj == 2u ? tthr[2] : tthr[3]));
          take = d2 < tt && (w & kIdMask) - mstart >= bpm;
        } else {
          take = d2 < thr;
        }
        take = take && u < rem;
        kid[min(row0 + tk, kmax + 1) * kNlistBlock + lane] = (code_t)(t + u);
        tk += take ? 1 : 0;
      }
      cnt += tk;
    };
    // slots [b, e) of a column whose candidate numbers are slot + o; f0..f3:
    // the records of slots b .. b+3, loaded ahead.  Two batches of four in
    // flight, in alternating registers; a batch loads only after one with
    // candidates left, so the reads stop 7 records past e (the record array
    // is padded for that)
    auto scan = [&](uint32_t b, uint32_t e, uint32_t o, float4 f0, float4 f1, float4 f2, float4 f3) {
      if (b >= e) return;
      const float4* q = PK + b;
      float4 ra[4] = {f0, f1, f2, f3}, rb4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) rb4[u] = q[4 + u];
      int rem = (int)(e - b);
      uint32_t t = b + o;
      while (true) {
        test4(ra, rem, t);
        rem -= 4;
        if (rem <= 0) break;
        q += 8;
#pragma unroll
        for (int u = 0; u < 4; ++u) ra[u] = q[u];
        test4(rb4, rem, t + 4u);
        rem -= 4;
        if (rem <= 0) break;
#pragma unroll
        for (int u = 0; u < 4; ++u) rb4[u] = q[4 + u];
        t += 8u;
      }
    };
    // the 9 columns, unrolled (their runs stay in registers)
#pragma unroll
    for (int col = 0; col < 9; ++col) {
      if (re[col] > rb[col]) {
        uint32_t o = 0u - span_lo;  // (mod 2^32)
        if (!by_span) {
          const int h = column_slot(ckey, column_key(J, cx, cy, col));
          o = coff[h];
        }
        scan(rb[col], re[col], o, PK[rb[col]], PK[rb[col] + 1], PK[rb[col] + 2], PK[rb[col] + 3]);
      }
    }
    if (wrap) {
      // the second z-runs (periodic z, a cell at either end)
      uint32_t b1[9], e1[9];
      column_runs9(B, J, cx, cy, za1, zb1, b1, e1);
      for (int col = 0; col < 9; ++col) {
        if (e1[col] <= b1[col]) continue;
        uint32_t o = 0u - span_lo;
        if (!by_span) {
          const int h = column_slot(ckey, column_key(J, cx, cy, col));
          o = coff[h];
        }
        scan(b1[col], e1[col], o, PK[b1[col]], PK[b1[col] + 1], PK[b1[col] + 2], PK[b1[col] + 3]);
      }
    }
  }
  // 3. the halo: kept candidates outside the tile, marked in the bitmap,
  // ranked in candidate order.  Codes of own-tile slots become kOwn | local
  // index; the lane's own slot (found by the walk unless the molecule rule
  // left it out) leaves the list, the last entry taking its place.
  // number of the tile's first slot (its slots have consecutive numbers)
  uint32_t t0 = first_local - span_lo;
  if (!by_span && valid) {
    const int h = column_slot(ckey, column_key(J, cx, cy, 4));  // the lane's own column
    t0 = coff[h] + first_local;
  }
  int nall = valid ? min(cnt, kmax + 1) : 0;
  int pself = -1;
  for (int k = 0; k < nall; k += kRow) {
    // eight codes read together (rows past the list read the last row, in bounds)
    uint32_t code[kRow];
#pragma unroll
    for (int u = 0; u < kRow; ++u) code[u] = (uint32_t)kid[min(k + u, kmax + kNlistRows - 1) * kNlistBlock + lane];
#pragma unroll
    for (int u = 0; u < kRow; ++u) {
      if (k + u >= nall) continue;
      const uint32_t loc = code[u] - t0;
      if (loc == (uint32_t)lane)
        pself = k + u;
      else if (loc < (uint32_t)kTile)
        kid[(k + u) * kNlistBlock + lane] = (code_t)(kOwn | loc);
      else
        atomicOr(&bits[code[u] >> 5], 1u << (code[u] & 31));
    }
  }
  if (pself >= 0) {
    kid[pself * kNlistBlock + lane] = kid[(nall - 1) * kNlistBlock + lane];
    nall -= 1;
  }
  const int found = valid ? cnt - (pself >= 0 ? 1 : 0) : 0;  // neighbours found
  const int stored = min(nall, kmax);
  // bead model: the molecule's beads id-2, id-1, id+1, id+2 (the bonded
  // terms' partners, which the lists leave out) found through the inverse
  // permutation, numbered like candidates (none when outside the tile's
  // candidates) and marked for the halo like list entries
  constexpr uint32_t kNoCode = 0xFFFFFFFFu;
  uint32_t pcode[4] = {kNoCode, kNoCode, kNoCode, kNoCode};
  if (typed && valid && bpm > 1u && !B.no_bw) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t g = myid - 2u + (uint32_t)(q < 2 ? q : q + 1);  // (wraps below 0: then outside)
      if (g - mstart >= bpm || g >= (uint32_t)J.n) continue;
      const uint32_t sl = B.INV[base + g];  // job-local slot
      uint32_t t = kNoCode;
      if (by_span) {
        if (sl >= span_lo && sl < span_hi) t = sl - span_lo;
      } else {
        // the hull holding the slot: ce, cb hold the hulls' first slots and
        // first numbers in slot order
        uint32_t lo = 0u, hi = nhull;
        while (hi - lo > 1u) {
          const uint32_t mid = (lo + hi) >> 1;
          if (ce[mid] <= sl)
            lo = mid;
          else
            hi = mid;
        }
        const uint32_t len = (lo + 1u < nhull ? cb[lo + 1u] : M) - cb[lo];
        if (nhull > 0u && sl >= ce[lo] && sl - ce[lo] < len) t = cb[lo] + (sl - ce[lo]);
      }
      if (t == kNoCode) continue;
      const uint32_t loc = t - t0;
      if (loc < (uint32_t)kTile) {
        pcode[q] = kOwn | loc;
      } else {
        atomicOr(&bits[t >> 5], 1u << (t & 31));
        pcode[q] = t;
      }
    }
  }
  __syncthreads();
  uint32_t H = 0u;
  {
    const int w0 = 2 * lane;
    const uint32_t p0 = __popc(bits[w0]), p1 = __popc(bits[w0 + 1]);
    const uint32_t ex = block_scan(p0 + p1, scan_sh, H);
    wpre[w0] = ex;
    wpre[w0 + 1] = ex + p0;
  }
  __syncthreads();
  const uint32_t hcap = (uint32_t)B.hcap;
  // the halo list: each lane takes bitmap words and writes their set bits
  for (uint32_t wi = lane; wi < (M + 31u) / 32u; wi += kNlistBlock) {
    uint32_t w = bits[wi];
    // by columns: the hull holding the word's first bit, found once per word
    // (later bits of the word step forward from it)
    uint32_t h = 0u;
    if (!by_span && w != 0u) {
      uint32_t lo = 0u, hi = nhull;
      while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (cb[mid] <= wi * 32u)  // cb: the hulls' first numbers in slot order
          lo = mid;
        else
          hi = mid;
      }
      h = lo;
    }
    for (uint32_t rank = wpre[wi]; w != 0u && rank < hcap; ++rank, w &= w - 1u) {
      const uint32_t t = wi * 32u + (uint32_t)(__ffs(w) - 1);
      uint32_t slot = span_lo + t;
      if (!by_span) {
        while (h + 1 < nhull && cb[h + 1] <= t) ++h;
        slot = ce[h] + (t - cb[h]);  // ce: the hulls' first slots in slot order
      }
      B.HALO[gt * (int64_t)hcap + rank] = (uint32_t)(base + slot);
      if (kWide) wrec[kTile + rank] = __float_as_uint(PK[slot].w);
    }
  }
  if (lane == 0) {
    B.HCNT[gt] = H;
    // a halo beyond the capacity stops the job before its first step on these lists
    if (H > hcap) atomicMin(&K.stop_at, (long long)J.step0);
  }
  if (kWide) __syncthreads();  // the window's records
  // record word of window entry e (clamped: a halo beyond the capacity stops
  // the job, its entries are never used)
  auto rec = [&](uint32_t e) { return wrec[min(e, wlen - 1u)]; };
  if (valid) {
    // the window entries of codes k .. k+7, without branches: the codes, then
    // their bitmap words and ranks (an own slot keeps its local index)
    auto entries = [&](int k, uint32_t* e) {
      uint32_t code[kRow], w[kRow], pre[kRow];
#pragma unroll
      for (int u = 0; u < kRow; ++u) {
        code[u] = (uint32_t)kid[min(k + u, kmax) * kNlistBlock + lane];
        if (k + u >= stored) code[u] = kOwn;  // past the list: entry 0
      }
#pragma unroll
      for (int u = 0; u < kRow; ++u) {
        const uint32_t v = code[u] & ~kOwn;
        w[u] = bits[v >> 5];
        pre[u] = wpre[v >> 5];
      }
#pragma unroll
      for (int u = 0; u < kRow; ++u) {
        const uint32_t v = code[u] & ~kOwn;
        e[u] = (code[u] & kOwn) ? v : (uint32_t)kTile + pre[u] + __popc(w[u] & ((1u << (v & 31)) - 1u));
      }
    };
    if (sorted) {
      // FP64 class: the entries in place, then the lane's list by particle
      // index (the order of the FP64 sums), insertion sort over its few entries
      for (int k = 0; k < stored; k += kRow) {
        uint32_t e[kRow];
        entries(k, e);
#pragma unroll
        for (int u = 0; u < kRow; ++u)
          if (k + u < stored) kid[(k + u) * kNlistBlock + lane] = (code_t)e[u];
      }
      const uint32_t idm = typed ? kIdMask : 0xFFFFFFFFu;
      for (int a = 1; a < stored; ++a) {
        const code_t c = kid[a * kNlistBlock + lane];
        const uint32_t key = rec(c) & idm;
        int b = a;
        for (; b > 0; --b) {
          const code_t prev = kid[(b - 1) * kNlistBlock + lane];
          if ((rec(prev) & idm) <= key) break;
          kid[b * kNlistBlock + lane] = prev;
        }
        kid[b * kNlistBlock + lane] = c;
      }
    }
    for (int k = 0; k < stored; k += kRow) {
      // the row's eight entries (FP64 class: already ordered)
      uint32_t e[kRow];
      if (sorted) {
#pragma unroll
        for (int u = 0; u < kRow; ++u) e[u] = (uint32_t)kid[min(k + u, kmax) * kNlistBlock + lane];
      } else {
        entries(k, e);
      }
#pragma unroll
      for (int u = 0; u < kRow; ++u) {
        uint32_t en = e[u];
        // bead model: the partner's type in the top bits
        if (typed) en |= (rec(en) >> kTypeShift) << kEntryTypeShift;
        e[u] = k + u < stored ? en & 0xFFFFu : 0u;
      }
      store_row<kStream>(B.NL, C, k, i, e);
    }
    B.NCNT[i] = (uint32_t)stored;
    if (typed) {
      // the bonded partners' window entries, with their types
      uint32_t pe[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t v = pcode[q] & ~kOwn;
        uint32_t en = (pcode[q] & kOwn) ? v
                                        : (uint32_t)kTile + wpre[v >> 5] + __popc(bits[v >> 5] & ((1u << (v & 31)) - 1u));
        en |= (rec(en) >> kTypeShift) << kEntryTypeShift;
        pe[q] = pcode[q] == kNoCode ? 0xFFFFu : en & 0xFFFFu;
      }
      B.BW[i] = make_uint2(pe[0] | (pe[1] << 16), pe[2] | (pe[3] << 16));
    }
  }
  // list statistics of these 64 slots (no atomics); an overflow stops the job
  // before its first step on these lists
  uint32_t mx = (uint32_t)found, sm = (uint32_t)stored;
  for (int o = 32; o > 0; o >>= 1) {
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    sm += (uint32_t)__shfl_xor((int)sm, o, 64);
  }
  const int64_t g0 = i - (lane % kGroup);
  if (lane % kGroup == 0 && g0 < J.off + J.n) {
    B.NLSTAT[2 * (g0 / kGroup)] = mx;
    B.NLSTAT[2 * (g0 / kGroup) + 1] = sm;
    if ((int)mx > kmax) atomicMin(&K.stop_at, (long long)J.step0);
  }
}

// Dynamic LDS of k_nlist for a list capacity kmax: the kept neighbours'
// 16-bit codes (room for kmax + 1 with the lane's own slot, and four rows for
// what does not fit), then table_words record words (the window's, in the
// wide instance, when they are staged in LDS).
constexpr size_t nlist_lds_bytes(int kmax, int64_t table_words) {
  return (size_t)(kmax + kNlistRows) * kNlistBlock * 2 + 4 * (size_t)table_words;
}

// Static LDS of k_nlist (column table, halo bitmap).
constexpr int64_t nlist_static_lds(bool) {
  return 4 * (4 * kColCap) + 8 * (kCandCap / 32) + 4 * (kNlistBlock / 64) + 16;
}

// Diagnostics of one job from the finish kernel's per-particle values (Section
// 3.1: K and U summed, constraint residuals maximised), in two passes with a
// fixed reduction tree, so the result depends only on n, not on scheduling.
// Pass 1: workgroup b reduces its contiguous chunk into part[4 b .. 4 b + 3];
// pass 2: one workgroup reduces the partials into out[0..3] = K, U, gdist_max,
// nv_max.
constexpr int kDiagThreads = 256;
constexpr int kDiagBlocks = 256;

__device__ __forceinline__ void diag_tree(double* sk, double* su, double* sg, double* sv, int tid) {
  for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
    __syncthreads();
    if (tid < w) {
      sk[tid] += sk[tid + w];
      su[tid] += su[tid + w];
      sg[tid] = fmax(sg[tid], sg[tid + w]);
      sv[tid] = fmax(sv[tid], sv[tid + w]);
    }
  }
  __syncthreads();
}

// One workgroup's share of the job's diagnostics: the n values from off split
// into nb equal pieces, piece b reduced over kDiagThreads threads.
__device__ __forceinline__ void diag_partial_block(const double* __restrict__ OD, int64_t C, int64_t off, int64_t n,
                                                   int nb, int b, double* __restrict__ part, double* sk, double* su,
                                                   double* sg, double* sv) {
  const int tid = threadIdx.x;
  const int64_t chunk = (n + nb - 1) / nb;
  const int64_t b0 = (int64_t)b * chunk, b1 = min(b0 + chunk, n);
  double k = 0.0, u = 0.0, g = 0.0, v = 0.0;
  for (int64_t i = b0 + tid; i < b1; i += kDiagThreads) {
    k += OD[off + i];
    u += OD[C + off + i];
    g = fmax(g, OD[2 * C + off + i]);
    v = fmax(v, OD[3 * C + off + i]);
  }
  sk[tid] = k, su[tid] = u, sg[tid] = g, sv[tid] = v;
  diag_tree(sk, su, sg, sv, tid);
  if (tid == 0) {
    double* o = part + 4 * b;
    o[0] = sk[0], o[1] = su[0], o[2] = sg[0], o[3] = sv[0];
  }
}

// The nb partials of a job reduced to its four results.
__device__ __forceinline__ void diag_final_block(const double* __restrict__ part, int nb, double* __restrict__ out,
                                                 double* sk, double* su, double* sg, double* sv) {
  const int tid = threadIdx.x;
  double k = 0.0, u = 0.0, g = 0.0, v = 0.0;
  for (int b = tid; b < nb; b += kDiagThreads) {
    k += part[4 * b];
    u += part[4 * b + 1];
    g = fmax(g, part[4 * b + 2]);
    v = fmax(v, part[4 * b + 3]);
  }
  sk[tid] = k, su[tid] = u, sg[tid] = g, sv[tid] = v;
  diag_tree(sk, su, sg, sv, tid);
  if (tid == 0) out[0] = sk[0], out[1] = su[0], out[2] = sg[0], out[3] = sv[0];
}

__global__ void __launch_bounds__(kDiagThreads) k_diag_partial(const double* __restrict__ OD, int64_t C, int64_t off,
                                                               int64_t n, double* __restrict__ part) {
  __shared__ double sk[kDiagThreads], su[kDiagThreads], sg[kDiagThreads], sv[kDiagThreads];
  diag_partial_block(OD, C, off, n, (int)gridDim.x, (int)blockIdx.x, part, sk, su, sg, sv);
}

__global__ void __launch_bounds__(kDiagThreads) k_diag_final(const double* __restrict__ part, int nb,
                                                             double* __restrict__ out) {
  __shared__ double sk[kDiagThreads], su[kDiagThreads], sg[kDiagThreads], sv[kDiagThreads];
  diag_final_block(part, nb, out, sk, su, sg, sv);
}

// Several jobs' diagnostics in one pair of launches (the same pieces and trees
// as one job at a time, so the same results): job q0 + blockIdx.y, its pieces
// in part + 4 kDiagBlocks (q0 + blockIdx.y).
struct DiagJob {
  int64_t off, n;
  int64_t nb;
};
__global__ void __launch_bounds__(kDiagThreads) k_diag_partial_many(const double* __restrict__ OD, int64_t C,
                                                                    const DiagJob* __restrict__ dj, int q0,
                                                                    double* __restrict__ part) {
  __shared__ double sk[kDiagThreads], su[kDiagThreads], sg[kDiagThreads], sv[kDiagThreads];
  const int q = q0 + (int)blockIdx.y;
  const DiagJob d = dj[q];
  if ((int64_t)blockIdx.x >= d.nb) return;
  diag_partial_block(OD, C, d.off, d.n, (int)d.nb, (int)blockIdx.x, part + (size_t)4 * kDiagBlocks * q, sk, su, sg,
                     sv);
}
__global__ void __launch_bounds__(kDiagThreads) k_diag_final_many(const double* __restrict__ part,
                                                                  const DiagJob* __restrict__ dj,
                                                                  double* __restrict__ out) {
  __shared__ double sk[kDiagThreads], su[kDiagThreads], sg[kDiagThreads], sv[kDiagThreads];
  const int q = (int)blockIdx.x;
  if (dj[q].n <= 0) return;
  diag_final_block(part + (size_t)4 * kDiagBlocks * q, (int)dj[q].nb, out + 4 * q, sk, su, sg, sv);
}

// Positions and momenta of several jobs (finish outputs, by particle index)
// packed one after another for one copy to the host: job q0 + blockIdx.y's
// 3n values of OX at dst + at, then its 3n values of OP.
struct PackJob {
  int64_t off, n, at;
};
__global__ void __launch_bounds__(256) k_pack_xp(const double* __restrict__ OX, const double* __restrict__ OP,
                                                 const PackJob* __restrict__ pj, int q0, double* __restrict__ dst) {
  const PackJob p = pj[q0 + (int)blockIdx.y];
  const int64_t m = 3 * p.n;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
    dst[p.at + k] = OX[3 * p.off + k];
    dst[p.at + m + k] = OP[3 * p.off + k];
  }
}

// Per-job reductions read by the host after a chunk of steps: at the end of
// each chunk the largest per-tile displacement bound; after list builds only
// the list statistics (largest list, sum of list lengths, largest tile halo;
// the bound is read after the chunk that follows every build).  One workgroup
// per job record.
constexpr int kStatsThreads = 1024;
__global__ void __launch_bounds__(kStatsThreads) k_job_stats(DevBufs B, int with_lists) {
  __shared__ double ra[kStatsThreads / 64], rs[kStatsThreads / 64];
  __shared__ uint32_t rm[kStatsThreads / 64], rh[kStatsThreads / 64];
  const int job = blockIdx.x;
  const JobDev& J = B.jobs[job];
  if (J.n <= 0) return;
  double a = 0.0, sm = 0.0;
  uint32_t mx = 0u, hx = 0u;
  const int64_t g0 = J.off / kGroup, g1 = (J.off + J.n + kGroup - 1) / kGroup;
  // four independent loads in flight per thread (one workgroup serves a job)
  constexpr int64_t kStride = kStatsThreads;
  int64_t g = g0 + threadIdx.x;
  if (!with_lists) {
    for (; g + 3 * kStride < g1; g += 4 * kStride) {
      const double t0 = B.TACC[g], t1 = B.TACC[g + kStride], t2 = B.TACC[g + 2 * kStride], t3 = B.TACC[g + 3 * kStride];
      a = fmax(fmax(a, fmax(t0, t1)), fmax(t2, t3));
    }
    for (; g < g1; g += kStride) a = fmax(a, B.TACC[g]);
  } else {
    // list-length sums are integers: exact in FP64 in any order
    const uint2* __restrict__ st = reinterpret_cast<const uint2*>(B.NLSTAT);
    g = g0 + threadIdx.x;
    for (; g + 3 * kStride < g1; g += 4 * kStride) {
      const uint2 q0 = st[g], q1 = st[g + kStride], q2 = st[g + 2 * kStride], q3 = st[g + 3 * kStride];
      mx = max(mx, max(max(q0.x, q1.x), max(q2.x, q3.x)));
      sm += (double)q0.y + (double)q1.y + (double)q2.y + (double)q3.y;
    }
    for (; g < g1; g += kStride) {
      const uint2 q = st[g];
      mx = max(mx, q.x);
      sm += (double)q.y;
    }
    const int64_t t0 = J.off / kTile, t1 = (J.off + J.n + kTile - 1) / kTile;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += kStride) hx = max(hx, B.HCNT[t]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    a = fmax(a, __shfl_xor(a, o, 64));
    sm += __shfl_xor(sm, o, 64);
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    hx = max(hx, (uint32_t)__shfl_xor((int)hx, o, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) ra[w] = a, rs[w] = sm, rm[w] = mx, rh[w] = hx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kStatsThreads / 64; ++q) a = fmax(a, ra[q]), sm += rs[q], mx = max(mx, rm[q]), hx = max(hx, rh[q]);
    JobBook& K = B.book[job];
    if (with_lists) {
      K.nl_max = (int)mx;
      K.nl_sum = sm;
      K.halo_max = (int)hx;
    } else {
      K.a_now = a;
    }
  }
}

// ---------------------------------------------------------------------------
// Segmented exclusive scan, three passes.
// A chunk is a piece of one segment; chunks of a segment are consecutive in
// the chunk list.  Pass A scans each chunk (eight elements per thread, the
// thread totals by wavefront shuffles, the four wavefront totals through LDS)
// and writes its total; pass B scans the totals within each segment (one
// workgroup); pass C adds them.
// ---------------------------------------------------------------------------
struct Chunk {
  int64_t start;   // element index of the chunk's first element
  int len;         // elements in the chunk (<= kScanChunk)
  int seg_first;   // index (in the chunk list) of the segment's first chunk
};

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanChunk = kScanThreads * kScanPer;

template <bool kPopc>
__global__ void __launch_bounds__(kScanThreads) k_scan_a(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                         const Chunk* __restrict__ chunks, uint32_t* __restrict__ sums) {
  __shared__ uint32_t wtot[kScanThreads / 64];
  const Chunk ch = chunks[blockIdx.x];
  const int t = (int)threadIdx.x, wl = t & 63, w = t >> 6;
  // this thread's eight consecutive elements: two 16-byte loads when the
  // chunk starts on a 16-byte boundary (input and output share the offset)
  // and all eight are in the chunk, else one at a time
  const int i0 = t * kScanPer;
  const bool whole = i0 + kScanPer <= ch.len && (ch.start & 3) == 0;
  uint32_t v[kScanPer];
  if (whole) {
    const uint4 q0 = *reinterpret_cast<const uint4*>(in + ch.start + i0);
    const uint4 q1 = *reinterpret_cast<const uint4*>(in + ch.start + i0 + 4);
    v[0] = q0.x, v[1] = q0.y, v[2] = q0.z, v[3] = q0.w;
    v[4] = q1.x, v[5] = q1.y, v[6] = q1.z, v[7] = q1.w;
  } else {
#pragma unroll
    for (int e = 0; e < kScanPer; ++e) v[e] = i0 + e < ch.len ? in[ch.start + i0 + e] : 0u;
  }
  uint32_t run = 0;
#pragma unroll
  for (int e = 0; e < kScanPer; ++e) {
    const uint32_t a = kPopc ? (uint32_t)__popc(v[e]) : v[e];
    v[e] = run;
    run += a;
  }
  // inclusive scan of the thread totals within the wavefront, then across
  // the four wavefronts
  uint32_t incl = run;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = (uint32_t)__shfl_up((int)incl, o, 64);
    if (wl >= o) incl += u;
  }
  if (wl == 63) wtot[w] = incl;
  __syncthreads();
  uint32_t base = incl - run, total = 0u;
#pragma unroll
  for (int q = 0; q < kScanThreads / 64; ++q) {
    if (q < w) base += wtot[q];
    total += wtot[q];
  }
  if (whole) {
    *reinterpret_cast<uint4*>(out + ch.start + i0) = make_uint4(base + v[0], base + v[1], base + v[2], base + v[3]);
    *reinterpret_cast<uint4*>(out + ch.start + i0 + 4) = make_uint4(base + v[4], base + v[5], base + v[6], base + v[7]);
  } else {
#pragma unroll
    for (int e = 0; e < kScanPer; ++e)
      if (i0 + e < ch.len) out[ch.start + i0 + e] = base + v[e];
  }
  if (t == 0) sums[blockIdx.x] = total;
}

constexpr int kScanB = 1024;

// Segmented exclusive scan of the chunk totals in one workgroup, 1024 at a
// time, carrying the running total of the segment that crosses a tile edge.
__global__ void __launch_bounds__(kScanB) k_scan_b(uint32_t* __restrict__ sums, const Chunk* __restrict__ chunks,
                                                   int nchunks) {
  __shared__ uint32_t sv[kScanB];
  __shared__ int sf[kScanB];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0u;
  __syncthreads();
  for (int base = 0; base < nchunks; base += kScanB) {
    const int c = base + threadIdx.x;
    const bool in = c < nchunks;
    const uint32_t v = in ? sums[c] : 0u;
    const int head = in ? (chunks[c].seg_first == c) : 1;
    sv[threadIdx.x] = v;
    sf[threadIdx.x] = head;
    __syncthreads();
    for (int o = 1; o < kScanB; o <<= 1) {
      uint32_t av = 0u;
      int af = 0;
      const bool take = threadIdx.x >= o;
      if (take) {
        av = sv[threadIdx.x - o];
        af = sf[threadIdx.x - o];
      }
      __syncthreads();
      if (take && !sf[threadIdx.x]) sv[threadIdx.x] += av;
      if (take) sf[threadIdx.x] |= af;
      __syncthreads();
    }
    uint32_t incl = sv[threadIdx.x];
    if (!sf[threadIdx.x]) incl += carry;  // no segment start between the tile edge and here
    if (in) sums[c] = incl - v;
    __syncthreads();
    if (threadIdx.x == kScanB - 1) carry = incl;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_c(uint32_t* __restrict__ out, const Chunk* __restrict__ chunks,
                                                         const uint32_t* __restrict__ sums) {
  const Chunk ch = chunks[blockIdx.x];
  const uint32_t add = sums[blockIdx.x];
  if (add == 0u) return;
  for (int idx = threadIdx.x; idx < ch.len; idx += kScanThreads) out[ch.start + idx] += add;
}

// Passes B and C in one, for segments of at most kScanBcMax chunks: each
// workgroup sums the totals of the chunks before its own in its segment
// (integers: the same result in any order) and adds that to its chunk.
constexpr int kScanBcMax = 2048;
__global__ void __launch_bounds__(kScanThreads) k_scan_bc(uint32_t* __restrict__ out, const Chunk* __restrict__ chunks,
                                                          const uint32_t* __restrict__ sums) {
  __shared__ uint32_t red[kScanThreads / 64];
  const int c = (int)blockIdx.x;
  const Chunk ch = chunks[c];
  uint32_t a = 0u;
  for (int q = ch.seg_first + (int)threadIdx.x; q < c; q += kScanThreads) a += sums[q];
  for (int o = 32; o > 0; o >>= 1) a += (uint32_t)__shfl_xor((int)a, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  uint32_t add = 0u;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) add += red[w];
  if (add == 0u) return;
  for (int idx = threadIdx.x; idx < ch.len; idx += kScanThreads) out[ch.start + idx] += add;
}

}  // namespace mdk
