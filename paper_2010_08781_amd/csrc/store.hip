// store.hip -- the device graph store (in-memory CSR + CSC with 64-bit
// offsets, Section 4.2: vertices and adjacency lists in global arrays shared
// by all workers), its validation, the out-degrees used by broadcast
// (Section 3), and the pull-side tiling of the CSC.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.h"

namespace ipg {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
ipg_status fail(ipg_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}
ipg_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return IPG_EDEVICE;
}

__global__ void fill_u32_kernel(uint32_t* p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void fill_f64_kernel(double* p, uint64_t n, double v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
hipError_t fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, kBlock * 4, 8192)), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t fill_f64(double* p, uint64_t n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(n, kBlock * 4, 8192)), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}

enum : uint32_t { kFlagOffsets = 0, kFlagCsrIds = 1, kFlagCscIds = 2, kFlagDegree = 3, kNumFlags = 4 };

// off[0] == 0, non-decreasing, off[n] == e.
__global__ void validate_offsets_kernel(const uint64_t* off, uint32_t n, uint64_t e, uint32_t* flags) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += stride)
    if (off[v] > off[v + 1]) flags[kFlagOffsets] = 1;
  if (blockIdx.x == 0 && threadIdx.x == 0 && (off[0] != 0 || off[n] != e)) flags[kFlagOffsets] = 1;
}

__global__ void validate_ids_kernel(const int32_t* adj, uint64_t e, uint32_t n, uint32_t* flag) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < e; i += stride) {
    const int32_t x = adj[i];
    bad |= (x < 0) | (static_cast<uint32_t>(x) >= n);
  }
  if (__ballot(bad) && lane_id() == 0) *flag = 1;
}

__global__ void outdeg_kernel(const uint64_t* off, uint32_t n, uint32_t* outdeg, uint32_t* flags) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const uint64_t d = off[v + 1] - off[v];
    if (d > 0xFFFFFFFFull) flags[kFlagDegree] = 1;
    outdeg[v] = static_cast<uint32_t>(d);
  }
}

// Pull row-groups: group k holds the rows whose first in-edge lies in
// [k*T, (k+1)*T), i.e. pull_rb[k] = first row v with off[v] >= k*T.  Row v
// owns the groups k in (off[v-1]/T, off[v]/T]; v = n owns the tail.
__global__ void pull_groups_kernel(const uint64_t* off, uint32_t n, uint32_t nb, uint32_t* rb) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v <= n; v += stride) {
    const uint64_t lo = v == 0 ? 0 : off[v - 1] / kPullTile + 1;
    uint64_t hi = off[v] / kPullTile;
    if (hi > (uint64_t)nb - 1) hi = (uint64_t)nb - 1;
    for (uint64_t k = lo; k <= hi; ++k) rb[k] = static_cast<uint32_t>(v);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) rb[nb] = n;
}

__global__ void long_rows_kernel(const uint64_t* off, uint32_t n, uint32_t* list, uint32_t cap, uint32_t* count) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v0 = blockIdx.x * (uint64_t)blockDim.x; v0 < n; v0 += stride) {
    const uint64_t v = v0 + threadIdx.x;
    const bool pred = v < n && off[v + 1] - off[v] > kPullTile;
    const uint64_t mask = __ballot(pred);
    if (mask == 0) continue;
    const uint32_t leader = static_cast<uint32_t>(__ffsll(static_cast<unsigned long long>(mask)) - 1);
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(count, static_cast<uint32_t>(__popcll(mask)));
    base = __shfl(base, static_cast<int>(leader));
    const uint32_t slot = base + lanes_below(mask);
    if (pred && slot < cap) list[slot] = static_cast<uint32_t>(v);
  }
}

// Edge ranges of the pull items (row pieces: [off[r0], off[r1]); chunks:
// kWaveTile in-edges of row r0 starting at chunk index e0 * kWaveTile).
__global__ void item_edges_kernel(const uint64_t* off, PullItem* items, uint32_t ni) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < ni; i += (uint64_t)gridDim.x * blockDim.x) {
    PullItem it = items[i];
    if (it.slot == kNoSlot) {
      it.e0 = off[it.r0];
      it.ne = static_cast<uint32_t>(off[it.r1] - it.e0);
    } else {
      const uint64_t beg = off[it.r0] + it.e0 * kWaveTile, end = off[it.r0 + 1];
      it.e0 = beg;
      it.ne = static_cast<uint32_t>(end - beg < kWaveTile ? end - beg : kWaveTile);
    }
    items[i] = it;
  }
}

__global__ void row_degrees_kernel(const uint64_t* off, const uint32_t* rows, uint32_t nr, uint64_t* deg) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nr; i += (uint64_t)gridDim.x * blockDim.x)
    deg[i] = off[rows[i] + 1] - off[rows[i]];
}


// Hot-first CSC: row v of the caller's CSC becomes row perm[v], its
// sources renamed, in their original order (one wavefront per row).
__global__ void rename_rows_kernel(const uint64_t* off, const int32_t* src, uint32_t n, const uint32_t* perm,
                                   const uint64_t* off_hot, int32_t* src_hot) {
  const uint64_t nw = (uint64_t)gridDim.x * blockDim.x / kWave;
  for (uint64_t v = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / kWave; v < n; v += nw) {
    const uint64_t b = off[v], d = off[v + 1] - b, h = off_hot[perm[v]];
    for (uint64_t j = lane_id(); j < d; j += kWave) src_hot[h + j] = static_cast<int32_t>(perm[src[b + j]]);
  }
}

// out[perm[v]] = in[v].
__global__ void scatter_u32_kernel(const uint32_t* in, const uint32_t* perm, uint32_t n, uint32_t* out) {
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x)
    out[perm[v]] = in[v];
}

static void carve_tiling(Carver& c, uint32_t n, uint64_t e, TilingTables* t) {
  t->pull_rb = c.take<uint32_t>(num_pull_groups(e) + 1);
  t->long_rows = c.take<uint32_t>(long_rows_cap(e));
  t->lr_first = c.take<uint32_t>(long_rows_cap(e) + 1);
  t->ch_row = c.take<uint32_t>(chunks_cap(e));
  t->items = c.take<PullItem>(items_cap(n, e));
  t->nb = t->nl = t->nc = t->ni = 0;
}

// Whether a blocked store also holds the blocked in-edges of the caller's
// CSC (blk_ids): with a hot-first store, for CC/SSSP, which keep the caller's
// names -- but not when it is symmetric: CC and SSSP then run under the new
// names on the hot-first table (min_space), whose hot sources are the
// most-read ones.
static bool ids_table(uint32_t flags) { return (flags & IPG_GRAPH_RENAME) && !(flags & IPG_GRAPH_SYMMETRIC); }

static size_t carve_graph(Carver& c, uint32_t n, uint64_t e, uint32_t flags, GraphTables* t) {
  GraphTables tt{};
  tt.outdeg = c.take<uint32_t>(n ? n : 1);
  tt.flags = c.take<uint32_t>(kNumFlags + 1);  // + long-row counter
  carve_tiling(c, n, e, &tt.pull);
  if (flags & IPG_GRAPH_RENAME) {
    tt.perm = c.take<uint32_t>(n ? n : 1);
    tt.iperm = c.take<uint32_t>(n ? n : 1);
    tt.outdeg_hot = c.take<uint32_t>(n ? n : 1);
    tt.off_hot = c.take<uint64_t>((size_t)n + 1);
    tt.src_hot = c.take<int32_t>(e ? e : 1);
    carve_tiling(c, n, e, &tt.pull_hot);
  }
  auto carve_blocked = [&](BlockedTables& b, bool binned) {
    b.edges = c.take<uint32_t>(e ? e : 1);
    b.chunks = c.take<BlkChunk>(binned ? bin_chunks_cap(n, e) : blk_chunks_cap(n, e));
    b.slices = c.take<BlkSlice>(blk_blocks_cap(n, e) + blk_target_slices(e));
    b.groups = c.take<BlkGroup>(blk_groups_cap(n, e));
    b.partial = c.take<double>(blk_partial_cap(e));
    if (binned) {
      const uint64_t nw = bin_windows(n) + 1;
      b.slots = c.take<double>(bin_slots_cap(n, e) + 1);
      b.bin_src = c.take<uint16_t>(bin_slots_cap(n, e) + 1);
      b.bin_runs = c.take<BinRun>(bin_runs_cap(n, e) + 1);
      b.bin_wflat = c.take<uint64_t>(nw);
      b.bin_wrun = c.take<uint32_t>(nw);
      b.bin_wgroup = c.take<uint64_t>(nw);
      b.bin_group = c.take<uint32_t>(bin_groups_cap(n, e));
      b.bin_units = c.take<BinUnit>(bin_units_cap(n, e));
    }
  };
  if (flags & IPG_GRAPH_BLOCKED) {
    carve_blocked(tt.blk, (flags & IPG_GRAPH_BINNED) != 0);
    if (ids_table(flags)) carve_blocked(tt.blk_ids, (flags & IPG_GRAPH_BINNED) != 0);
  }
  if (t) *t = tt;
  return align_up(c.used, 256);
}

// Pull tiling of a CSC (validated offsets): row-groups, long rows cut into
// chunks, and the work items.  `counter` is one device word of scratch.
static ipg_status build_tiling(const uint64_t* csc_off, uint32_t n, uint64_t e, TilingTables* t, uint32_t* counter,
                               hipStream_t s) {
  const uint32_t nb = num_pull_groups(e);
  const uint32_t gv = grid_for(n + 1ull, kBlock, 16384);
  IPG_HIP(fill_u32(counter, 1, 0, s));
  hipLaunchKernelGGL(pull_groups_kernel, dim3(gv), dim3(kBlock), 0, s, csc_off, n, nb, t->pull_rb);
  IPG_HIP(hipGetLastError());
  const uint32_t cap = static_cast<uint32_t>(long_rows_cap(e));
  hipLaunchKernelGGL(long_rows_kernel, dim3(gv), dim3(kBlock), 0, s, csc_off, n, t->long_rows, cap, counter);
  IPG_HIP(hipGetLastError());
  uint32_t nl = 0;
  IPG_HIP(hipMemcpyAsync(&nl, counter, sizeof(nl), hipMemcpyDeviceToHost, s));
  IPG_HIP(hipStreamSynchronize(s));
  if (nl > cap) return fail(IPG_EBADGRAPH, "in-degree table overflow (offsets inconsistent with E)");
  uint32_t nc = 0;
  std::vector<uint32_t> lrows(nl), lfirst(nl + 1, 0);
  if (nl > 0) {
    // Long rows in ascending order (a deterministic assignment to
    // workgroups), cut into chunks of kWaveTile in-edges.
    IPG_HIP(hipMemcpyAsync(lrows.data(), t->long_rows, nl * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    IPG_HIP(hipStreamSynchronize(s));
    std::sort(lrows.begin(), lrows.end());
    IPG_HIP(hipMemcpyAsync(t->long_rows, lrows.data(), nl * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    // degrees via the item table's space (24 bytes per item, more items than long rows)
    uint64_t* degs = reinterpret_cast<uint64_t*>(t->items);
    hipLaunchKernelGGL(row_degrees_kernel, dim3(grid_for(nl, kBlock, 1024)), dim3(kBlock), 0, s, csc_off, t->long_rows,
                       nl, degs);
    IPG_HIP(hipGetLastError());
    std::vector<uint64_t> deg(nl);
    IPG_HIP(hipMemcpyAsync(deg.data(), degs, nl * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    IPG_HIP(hipStreamSynchronize(s));
    std::vector<uint32_t> chrow;
    uint64_t acc = 0;
    for (uint32_t l = 0; l < nl; ++l) {
      lfirst[l] = static_cast<uint32_t>(acc);
      const uint64_t k = (deg[l] + kWaveTile - 1) / kWaveTile;
      acc += k;
      if (acc > chunks_cap(e)) return fail(IPG_EBADGRAPH, "long-row chunk table overflow (offsets inconsistent with E)");
      for (uint64_t j = 0; j < k; ++j) chrow.push_back(l);
    }
    lfirst[nl] = static_cast<uint32_t>(acc);
    nc = static_cast<uint32_t>(acc);
    IPG_HIP(hipMemcpyAsync(t->lr_first, lfirst.data(), (nl + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    IPG_HIP(hipMemcpyAsync(t->ch_row, chrow.data(), nc * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    IPG_HIP(hipStreamSynchronize(s));
  }
  // Pull work items: the long-row chunks, then each row-group cut into
  // pieces of at most kItemRows rows (a group's long last row is chunked).
  std::vector<uint32_t> rb(nb + 1);
  IPG_HIP(hipMemcpyAsync(rb.data(), t->pull_rb, (nb + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  IPG_HIP(hipStreamSynchronize(s));
  std::vector<PullItem> items;
  items.reserve(static_cast<size_t>(nb) + nc + n / kItemRows + 1);
  for (uint32_t l = 0; l < nl; ++l)
    for (uint32_t j = lfirst[l]; j < lfirst[l + 1]; ++j)
      items.push_back(PullItem{j - lfirst[l], 0, lrows[l], lrows[l] + 1, j});
  for (uint32_t k = 0; k < nb; ++k) {
    const uint32_t r0 = rb[k];
    uint32_t r1 = rb[k + 1];
    if (r1 > r0 && std::binary_search(lrows.begin(), lrows.end(), r1 - 1)) --r1;
    for (uint32_t a = r0; a < r1; a += kItemRows) items.push_back(PullItem{0, 0, a, std::min(r1, a + kItemRows), kNoSlot});
  }
  if (items.size() > items_cap(n, e)) return fail(IPG_EBADGRAPH, "pull item table overflow");
  const uint32_t ni = static_cast<uint32_t>(items.size());
  if (ni) {
    IPG_HIP(hipMemcpyAsync(t->items, items.data(), ni * sizeof(PullItem), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(item_edges_kernel, dim3(grid_for(ni, kBlock, 4096)), dim3(kBlock), 0, s, csc_off, t->items, ni);
    IPG_HIP(hipGetLastError());
    IPG_HIP(hipStreamSynchronize(s));
  }
  t->nb = nb;
  t->nl = nl;
  t->nc = nc;
  t->ni = ni;
  return IPG_OK;
}

// The hot-first store: names by descending out-degree (degrees above 65534
// tie; ties in id order -- a counting sort on the host), the CSC rebuilt
// under those names and its tiling.
static ipg_status build_hot_store(const uint64_t* csc_off, const int32_t* csc_src, uint32_t n, uint64_t e,
                                  GraphTables* t, std::vector<uint32_t>& perm, hipStream_t s) {
  std::vector<uint32_t> deg(n), iperm(n);
  perm.assign(n, 0);
  IPG_HIP(hipMemcpyAsync(deg.data(), t->outdeg, n * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  std::vector<uint64_t> off((size_t)n + 1), off_hot((size_t)n + 1, 0);
  IPG_HIP(hipMemcpyAsync(off.data(), csc_off, off.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  IPG_HIP(hipStreamSynchronize(s));
  constexpr uint32_t kKeys = 1u << 16;
  std::vector<uint64_t> start(kKeys + 1, 0);
  auto key = [&](uint32_t v) { return kKeys - 1 - std::min<uint32_t>(deg[v], kKeys - 1); };
  for (uint32_t v = 0; v < n; ++v) ++start[key(v) + 1];
  for (uint32_t k = 0; k < kKeys; ++k) start[k + 1] += start[k];
  for (uint32_t v = 0; v < n; ++v) perm[v] = static_cast<uint32_t>(start[key(v)]++);
  for (uint32_t v = 0; v < n; ++v) iperm[perm[v]] = v;
  for (uint32_t v = 0; v < n; ++v) off_hot[(size_t)perm[v] + 1] = off[v + 1] - off[v];
  for (uint32_t r = 0; r < n; ++r) off_hot[(size_t)r + 1] += off_hot[r];
  IPG_HIP(hipMemcpyAsync(t->perm, perm.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, s));
  IPG_HIP(hipMemcpyAsync(t->iperm, iperm.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, s));
  IPG_HIP(hipMemcpyAsync(t->off_hot, off_hot.data(), off_hot.size() * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  const uint32_t gv = grid_for(n, kBlock, 16384);
  hipLaunchKernelGGL(scatter_u32_kernel, dim3(gv), dim3(kBlock), 0, s, t->outdeg, t->perm, n, t->outdeg_hot);
  IPG_HIP(hipGetLastError());
  if (e) {
    hipLaunchKernelGGL(rename_rows_kernel, dim3(grid_for(n, kWavesPerBlock, 16384)), dim3(kBlock), 0, s, csc_off,
                       csc_src, n, t->perm, t->off_hot, t->src_hot);
    IPG_HIP(hipGetLastError());
  }
  IPG_HIP(hipStreamSynchronize(s));
  return build_tiling(t->off_hot, n, e, &t->pull_hot, t->flags + kNumFlags, s);
}

// The blocked in-edges of a CSC (validated or not): built on the host
// (blocked_layout.h) and copied to the device tables.
static ipg_status build_blocked(const uint64_t* csc_off, const int32_t* csc_src, uint32_t n, uint64_t e,
                                BlockedTables* b, uint32_t hot, hipStream_t s) {
  std::vector<uint64_t> off((size_t)n + 1);
  std::vector<int32_t> src(e);
  IPG_HIP(hipMemcpyAsync(off.data(), csc_off, off.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  if (e) IPG_HIP(hipMemcpyAsync(src.data(), csc_src, e * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  IPG_HIP(hipStreamSynchronize(s));
  BlockedLayout L;
  if (const char* msg = blocked_layout(n, e, off.data(), src.data(), &L, hot)) return fail(IPG_EBADGRAPH, msg);
  std::vector<int32_t>().swap(src);
  if (e) IPG_HIP(hipMemcpyAsync(b->edges, L.packed.data(), e * sizeof(uint32_t), hipMemcpyHostToDevice, s));
  if (!L.chunks.empty())
    IPG_HIP(hipMemcpyAsync(b->chunks, L.chunks.data(), L.chunks.size() * sizeof(BlkChunk), hipMemcpyHostToDevice, s));
  if (!L.slices.empty())
    IPG_HIP(hipMemcpyAsync(b->slices, L.slices.data(), L.slices.size() * sizeof(BlkSlice), hipMemcpyHostToDevice, s));
  if (!L.groups.empty())
    IPG_HIP(hipMemcpyAsync(b->groups, L.groups.data(), L.groups.size() * sizeof(BlkGroup), hipMemcpyHostToDevice, s));
  b->hot = L.hot;
  b->bin_w0 = L.bin_w0;
  b->bin_nwin = L.hot ? static_cast<uint32_t>(L.bin_wflat.size() - 1) : 0u;
  b->nslots = L.nslots;
  if (L.hot) {
    auto put = [&](void* dst, const void* src_, size_t bytes) -> hipError_t {
      return bytes ? hipMemcpyAsync(dst, src_, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    IPG_HIP(put(b->bin_src, L.bin_src.data(), L.bin_src.size() * sizeof(uint16_t)));
    IPG_HIP(put(b->bin_runs, L.bin_runs.data(), L.bin_runs.size() * sizeof(BinRun)));
    IPG_HIP(put(b->bin_wflat, L.bin_wflat.data(), L.bin_wflat.size() * sizeof(uint64_t)));
    IPG_HIP(put(b->bin_wrun, L.bin_wrun.data(), L.bin_wrun.size() * sizeof(uint32_t)));
    IPG_HIP(put(b->bin_wgroup, L.bin_wgroup.data(), L.bin_wgroup.size() * sizeof(uint64_t)));
    IPG_HIP(put(b->bin_group, L.bin_group.data(), L.bin_group.size() * sizeof(uint32_t)));
    IPG_HIP(put(b->bin_units, L.bin_units.data(), L.bin_units.size() * sizeof(BinUnit)));
  }
  b->bin_nunits = static_cast<uint32_t>(L.bin_units.size());
  IPG_HIP(hipStreamSynchronize(s));
  b->nchunks = static_cast<uint32_t>(L.chunks.size());
  b->nslices = static_cast<uint32_t>(L.slices.size());
  b->ngroups = static_cast<uint32_t>(L.groups.size());
  return IPG_OK;
}

}  // namespace ipg

using namespace ipg;

extern "C" size_t ipg_graph_workspace_bytes(uint32_t num_vertices, uint64_t num_edges, uint32_t flags) {
  Carver c(nullptr);
  return carve_graph(c, num_vertices, num_edges, flags, nullptr);
}

extern "C" ipg_status ipg_graph_create(const ipg_graph_desc* d, void* ws, size_t ws_bytes, void* hip_stream,
                                       ipg_graph** out) {
  if (!out) return fail(IPG_EINVAL, "ipg_graph_create: out is NULL");
  *out = nullptr;
  if (!d) return fail(IPG_EINVAL, "ipg_graph_create: desc is NULL");
  const uint32_t n = d->num_vertices;
  const uint64_t e = d->num_edges;
  if (n == 0) return fail(IPG_EINVAL, "ipg_graph_create: num_vertices must be >= 1");
  if (n >= 0x80000000u) return fail(IPG_EINVAL, "ipg_graph_create: num_vertices must be < 2^31");
  const bool sym = d->flags & IPG_GRAPH_SYMMETRIC;
  const uint64_t* csc_off = d->csc_off ? d->csc_off : (sym ? d->csr_off : nullptr);
  const int32_t* csc_src = d->csc_src ? d->csc_src : (sym ? d->csr_dst : nullptr);
  const uint32_t* csc_w = d->csc_w ? d->csc_w : (sym ? d->csr_w : nullptr);
  if (!d->csr_off || !csc_off) return fail(IPG_EINVAL, "ipg_graph_create: offsets pointer is NULL");
  if (e > 0 && (!d->csr_dst || !csc_src)) return fail(IPG_EINVAL, "ipg_graph_create: adjacency pointer is NULL");
  if ((d->csr_w == nullptr) != (csc_w == nullptr))
    return fail(IPG_EINVAL, "ipg_graph_create: give weights for both CSR and CSC or for neither");
  const size_t need = ipg_graph_workspace_bytes(n, e, d->flags);
  if (!ws || ws_bytes < need)
    return fail(IPG_EWORKSPACE, "ipg_graph_create: graph workspace needs " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(ws) % 256)
    return fail(IPG_EWORKSPACE, "ipg_graph_create: workspace must be 256-byte aligned");

  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Carver c(ws);
  GraphTables t;
  carve_graph(c, n, e, d->flags, &t);

  IPG_HIP(fill_u32(t.flags, kNumFlags + 1, 0, s));
  const uint32_t gv = grid_for(n + 1ull, kBlock, 16384), ge = grid_for(e, kBlock * 8, 16384);
  if (d->flags & IPG_GRAPH_VALIDATE) {
    hipLaunchKernelGGL(validate_offsets_kernel, dim3(gv), dim3(kBlock), 0, s, d->csr_off, n, e, t.flags);
    IPG_HIP(hipGetLastError());
    if (e) hipLaunchKernelGGL(validate_ids_kernel, dim3(ge), dim3(kBlock), 0, s, d->csr_dst, e, n, t.flags + kFlagCsrIds);
    IPG_HIP(hipGetLastError());
    if (csc_off != d->csr_off || csc_src != d->csr_dst) {
      uint32_t* f2 = t.flags + kFlagCscIds;
      hipLaunchKernelGGL(validate_offsets_kernel, dim3(gv), dim3(kBlock), 0, s, csc_off, n, e, f2 - kFlagOffsets);
      IPG_HIP(hipGetLastError());
      if (e) hipLaunchKernelGGL(validate_ids_kernel, dim3(ge), dim3(kBlock), 0, s, csc_src, e, n, f2);
      IPG_HIP(hipGetLastError());
    }
    uint32_t h[kNumFlags];
    IPG_HIP(hipMemcpyAsync(h, t.flags, sizeof(h), hipMemcpyDeviceToHost, s));
    IPG_HIP(hipStreamSynchronize(s));
    if (h[kFlagOffsets]) return fail(IPG_EBADGRAPH, "offsets: off[0] != 0, off[N] != E or decreasing");
    if (h[kFlagCsrIds]) return fail(IPG_EBADGRAPH, "CSR destination id outside [0, N)");
    if (h[kFlagCscIds]) return fail(IPG_EBADGRAPH, "CSC source id outside [0, N), or CSC offsets invalid");
  }
  hipLaunchKernelGGL(outdeg_kernel, dim3(gv), dim3(kBlock), 0, s, d->csr_off, n, t.outdeg, t.flags);
  IPG_HIP(hipGetLastError());
  uint32_t h[kNumFlags];
  IPG_HIP(hipMemcpyAsync(h, t.flags, sizeof(h), hipMemcpyDeviceToHost, s));
  IPG_HIP(hipStreamSynchronize(s));
  if (h[kFlagDegree]) return fail(IPG_EBADGRAPH, "an out-degree exceeds 2^32-1");
  ipg_status rc = build_tiling(csc_off, n, e, &t.pull, t.flags + kNumFlags, s);
  if (rc != IPG_OK) return rc;
  std::vector<uint32_t> perm_host;
  if (d->flags & IPG_GRAPH_RENAME) {
    rc = build_hot_store(csc_off, csc_src, n, e, &t, perm_host, s);
    if (rc != IPG_OK) return rc;
  }
  if (d->flags & IPG_GRAPH_BLOCKED) {
    const uint32_t hot = (d->flags & IPG_GRAPH_BINNED) ? (d->binned_hot ? d->binned_hot : kBinHotDefault) : 0u;
    if (d->flags & IPG_GRAPH_RENAME) {
      rc = build_blocked(t.off_hot, t.src_hot, n, e, &t.blk, hot, s);
      if (rc == IPG_OK && ids_table(d->flags)) rc = build_blocked(csc_off, csc_src, n, e, &t.blk_ids, hot, s);
    } else {
      rc = build_blocked(csc_off, csc_src, n, e, &t.blk, hot, s);
    }
    if (rc != IPG_OK) return rc;
  }

  ipg_graph* g = new (std::nothrow) ipg_graph();
  if (!g) return fail(IPG_EINVAL, "ipg_graph_create: out of host memory");
  g->n = n;
  g->e = e;
  g->flags = d->flags | (csc_off == d->csr_off && csc_src == d->csr_dst ? IPG_GRAPH_SYMMETRIC : 0u);
  g->csr_off = d->csr_off;
  g->csr_dst = d->csr_dst;
  g->csc_off = csc_off;
  g->csc_src = csc_src;
  g->csr_w = d->csr_w;
  g->csc_w = csc_w;
  g->t = t;
  g->perm_host.swap(perm_host);
  IPG_HIP(hipGetDevice(&g->device));
  g->has_values = 0;
  g->last_app = -1;
  g->last_values = nullptr;
  *out = g;
  set_error("");
  return IPG_OK;
}

extern "C" void ipg_graph_destroy(ipg_graph* g) {
  if (!g) return;
  if (g->pr_exec) (void)hipGraphExecDestroy(g->pr_exec);
  if (g->pr_graph) (void)hipGraphDestroy(g->pr_graph);
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  for (hipEvent_t ev : g->events) (void)hipEventDestroy(ev);
  if (g->mirror) (void)hipHostFree(g->mirror);
  delete g;
}

extern "C" const char* ipg_last_error(void) { return g_last_error.c_str(); }
