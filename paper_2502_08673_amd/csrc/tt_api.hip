// tt_api.hip -- host side of libtt.so: validation, layout, the planner
// (grouping, tiling, work queue), plan workspace, graph capture, the
// autotuner and the one-shot entry points declared in include/tt.h.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "tt_gd.h"
#include "tt_mlp.h"
#include "tt_internal.h"

using namespace tt;

namespace {

thread_local int g_last_hip = 0;

#define TT_HIP(expr)                    \
  do {                                  \
    hipError_t e_ = (expr);             \
    if (e_ != hipSuccess) {             \
      g_last_hip = (int)e_;             \
      return TT_EHIP;                   \
    }                                   \
  } while (0)

#define TT_TRY(expr)       \
  do {                     \
    int s_ = (expr);       \
    if (s_ != TT_OK) return s_; \
  } while (0)

#ifndef TT_KERNEL_SIG
#define TT_KERNEL_SIG 0ull  // the build passes a hash of the enumeration kernel sources
#endif

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// ------------------------------------------------------------------ device
struct DevInfo {
  int ok = -1;  // -1 unknown, 0 not gfx950, 1 gfx950
  int cus = 0;
};
std::mutex g_dev_mu;
std::map<int, DevInfo> g_dev;

int device_info(int* cus) {
  int dev = 0;
  TT_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_dev_mu);
  DevInfo& di = g_dev[dev];
  if (di.ok < 0) {
    hipDeviceProp_t prop;
    TT_HIP(hipGetDeviceProperties(&prop, dev));
    di.ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 0;
    di.cus = prop.multiProcessorCount;
  }
  if (cus) *cus = di.cus;
  return di.ok == 1 ? TT_OK : TT_ENOTSUP;
}

// -------------------------------------------------------------- validation
uint64_t words_of(int F, int b) {
  const int fb = F * b;
  return fb >= 6 ? (1ull << (fb - 6)) : 1ull;
}

int validate_one(const tt_neuron& d) {
  if (d.F < 1 || d.F > TT_MAX_F || d.b < 1 || d.b > TT_MAX_B || d.o < 1 || d.o > TT_MAX_O) return TT_EINVAL;
  if (d.act != TT_ACT_IDENTITY && d.act != TT_ACT_RELU) return TT_EINVAL;
  if (d.F * d.b > TT_MAX_FB) return TT_ERANGE;
  const int K = (1 << d.o) - 1;
  for (int k = 1; k < K; ++k)
    if (d.thr[k] < d.thr[k - 1]) return TT_EINVAL;
  return TT_OK;
}

int validate_all(const tt_neuron* h, int n) {
  if (n < 0) return TT_EINVAL;
  if (n > 0 && !h) return TT_EINVAL;
  for (int i = 0; i < n; ++i) TT_TRY(validate_one(h[i]));
  return TT_OK;
}

// Every neuron's o*W words inside [0, total_words), and no two overlap.
int validate_ranges(const tt_neuron* h, int n, uint64_t total_words) {
  std::vector<std::pair<uint64_t, uint64_t>> r(n);
  for (int i = 0; i < n; ++i) {
    const uint64_t len = (uint64_t)h[i].o * words_of(h[i].F, h[i].b);
    if (h[i].word_off > total_words || len > total_words - h[i].word_off) return TT_ERANGE;
    r[i] = {h[i].word_off, h[i].word_off + len};
  }
  std::sort(r.begin(), r.end());
  for (int i = 1; i < n; ++i)
    if (r[i].first < r[i - 1].second) return TT_EINVAL;
  return TT_OK;
}

// Entries reserved for a neuron's mask table: the low min(6, F*b) row bits
// have coefficients w_j * 2^(bit within digit); the sums span exactly
// sum |coefficient| + 1 values, plus the all-zero sentinel.
int lut_cap_of(const tt_neuron& d) {
  const int fb = d.F * d.b;
  const int low = fb < 6 ? fb : 6;
  int s = 0;
  for (int i = 0; i < low; ++i) s += std::abs((int)d.w[i / d.b]) << (i % d.b);
  return s + 2;
}

// ---------------------------------------------------------------- planner
struct Group {
  int item_begin = 0, item_end = 0;
  int neuron_begin = 0, neuron_end = 0;  // into group_neurons
  int wide_wb = 0;                       // > 0: enumerated by the wide kernel (log2 words per plane)
  int wide_lds = 0;                      // its largest mask table (entries)
  int wide_upw = 1;                      // 256-word units per wave
  int o = 1;
};

struct PlanHost {
  int n = 0;
  uint64_t total_words = 0;
  tt_tune tune{};
  unsigned flags = 0;
  std::vector<tt_neuron> desc;
  std::vector<uint64_t> lut_off;
  std::vector<int32_t> lut_cap;
  uint64_t lut_total = 0;
  int lut_chunks = 1;  // the largest mask table in 64-entry chunks
  std::vector<TileInfo> tiles;
  std::vector<int32_t> tile_neuron;
  std::vector<int32_t> tile_lds;  // [n] LDS entry base of the neuron's mask table in its tile
  std::vector<int32_t> tile_pos;  // [n] position in tile_neuron, -1 for wide-group neurons
  std::vector<int32_t> sup_lists;  // neurons for the support from parameters: small ranges first
  int64_t sup_small = 0;           // how many of them have sums spanning < 512 values
  std::vector<WorkItem> items;
  std::vector<Group> groups;
  std::vector<int32_t> group_neurons;
  std::vector<int32_t> large;  // neurons whose tables the support kernels take wave by wave
  long max_chunks = 1, max_items = 1;
};

// Neurons with more than kSmallTableWords words per plane.
// Also the most check items any of them has per check: 512-word chunks
// (near items, the histogram's units) and 64 x 2^c-word far items of the
// digits whose row bits reach 15 and up (c <= 3 bits per group).  Work
// units beyond these would find nothing to do.
void build_large_list(PlanHost& P) {
  // neurons for the support from parameters: those whose sums span fewer
  // than 512 values first (one wave each), then the others
  auto range_of = [&](const tt_neuron& d) {
    int R = 0;
    for (int j = 0; j < d.F; ++j) R += std::abs((int)d.w[j]) * ((1 << d.b) - 1);
    return R;
  };
  P.sup_lists.clear();
  for (int i = 0; i < P.n; ++i)
    if (range_of(P.desc[i]) < 512) P.sup_lists.push_back(i);
  P.sup_small = (int64_t)P.sup_lists.size();
  for (int i = 0; i < P.n; ++i)
    if (range_of(P.desc[i]) >= 512) P.sup_lists.push_back(i);
  P.large.clear();
  P.max_chunks = 1;
  P.max_items = 1;
  for (int i = 0; i < P.n; ++i) {
    const tt_neuron& d = P.desc[i];
    const uint64_t W = words_of(d.F, d.b);
    if (W <= (uint64_t)kSmallTableWords) continue;
    P.large.push_back(i);
    const long chunks = (long)std::max<uint64_t>(1, W / 512);
    P.max_chunks = std::max(P.max_chunks, chunks);
    P.max_items = std::max(P.max_items, chunks - 1);
    for (int j = 0; j < d.F; ++j)
      for (int s0 = std::max(j * d.b, 15); s0 < (j + 1) * d.b; s0 += 3) {
        const int c = std::min(3, (j + 1) * d.b - s0);
        P.max_items = std::max(P.max_items, (long)(W >> (6 + c)));
      }
  }
}

tt_tune default_tune() {
  tt_tune t;
  t.chunk_words = 4096;
  t.blocks_per_cu = 2;
  t.waves = 4;
  t.nontemporal = 1;
  t.tile_neurons = kTileM;
  return t;
}

int check_tune(const tt_tune& t) {
  // at most 2^16 words per item keeps a lane's 16-bit threshold counts exact
  if (t.chunk_words < kTileN || t.chunk_words % kTileN || t.chunk_words > (1 << 16)) return TT_EINVAL;
  if (t.blocks_per_cu < 1 || t.blocks_per_cu > 8) return TT_EINVAL;
  if (t.waves != 4 && t.waves != 8) return TT_EINVAL;
  if (t.tile_neurons != 8 && t.tile_neurons != 16 && t.tile_neurons != kTileM) return TT_EINVAL;
  return TT_OK;
}

void build_plan(PlanHost& P, bool persistent) {
  const int n = P.n;
  P.lut_off.resize(n);
  P.lut_cap.resize(n);
  uint64_t acc = 0;
  P.lut_chunks = 1;
  for (int i = 0; i < n; ++i) {
    P.lut_cap[i] = lut_cap_of(P.desc[i]);
    P.lut_chunks = std::max(P.lut_chunks, (P.lut_cap[i] + 63) / 64);
    P.lut_off[i] = acc;
    acc += (uint64_t)P.lut_cap[i];
  }
  P.lut_total = acc;

  // Group by (F, b, o) in first-seen order.
  std::map<std::tuple<int, int, int>, int> key_to_group;
  std::vector<std::vector<int>> members;
  for (int i = 0; i < n; ++i) {
    auto key = std::make_tuple((int)P.desc[i].F, (int)P.desc[i].b, (int)P.desc[i].o);
    auto it = key_to_group.find(key);
    int g;
    if (it == key_to_group.end()) {
      g = (int)members.size();
      key_to_group[key] = g;
      members.emplace_back();
    } else {
      g = it->second;
    }
    members[g].push_back(i);
  }

  P.tiles.clear();
  P.tile_neuron.clear();
  P.tile_lds.assign(n, 0);
  P.items.clear();
  P.groups.clear();
  P.group_neurons.clear();
  for (const auto& mem : members) {
    Group G;
    G.neuron_begin = (int)P.group_neurons.size();
    for (int i : mem) P.group_neurons.push_back(i);
    G.neuron_end = (int)P.group_neurons.size();
    G.item_begin = (int)P.items.size();
    const tt_neuron& d0 = P.desc[mem[0]];
    const uint64_t W = words_of(d0.F, d0.b);
    G.o = d0.o;
    if (W >= (1ull << kWideMinLog2)) {  // no tiles: one wave per 256 words
      G.wide_wb = d0.F * d0.b - 6;
      for (int i : mem) G.wide_lds = std::max(G.wide_lds, (int)P.lut_cap[i]);
      // blocks of the tuned number of waves; units per wave from the tuned
      // words per item: chunk_words / (256 * waves), a power of two in
      // [1, kWideMaxUpw] with waves * upw at most the neuron's units
      const int nw = P.tune.waves;
      int upw = 1;
      while (upw * 2 <= P.tune.chunk_words / (256 * nw) && upw * 2 <= kWideMaxUpw) upw *= 2;
      while (upw > 1 && nw * upw > (1 << (G.wide_wb - 8))) upw /= 2;
      G.wide_upw = upw;
      G.item_end = G.item_begin;
      P.groups.push_back(G);
      continue;
    }
    size_t pos = 0;
    while (pos < mem.size()) {
      TileInfo ti{};
      ti.first = (int32_t)P.tile_neuron.size();
      ti.W = (int32_t)W;
      ti.F = d0.F;
      ti.b = d0.b;
      ti.o = d0.o;
      int lds = 0, cnt = 0;
      while (pos < mem.size() && cnt < P.tune.tile_neurons) {
        const int c = P.lut_cap[mem[pos]];
        if (cnt > 0 && lds + c > kLutLdsEntries) break;
        P.tile_neuron.push_back(mem[pos]);
        P.tile_lds[mem[pos]] = lds;
        lds += c;
        ++cnt;
        ++pos;
      }
      for (int k = cnt; k < kTileM; ++k) P.tile_neuron.push_back(-1);
      ti.count = cnt;
      ti.lut_total = lds;
      const int tile_id = (int)P.tiles.size();
      P.tiles.push_back(ti);
      const uint64_t chunk = (uint64_t)P.tune.chunk_words;
      for (uint64_t h0 = 0; h0 < W; h0 += chunk) {
        WorkItem wi{};
        wi.tile = tile_id;
        wi.h0 = (int32_t)h0;
        wi.count = (int32_t)std::min<uint64_t>(chunk, W - h0);
        P.items.push_back(wi);
      }
    }
    G.item_end = (int)P.items.size();
    P.groups.push_back(G);
  }
  // Mask tables in tile order (each tile's back to back, as in its LDS copy),
  // then the wide groups' neurons; tile positions of the tile members.
  P.tile_pos.assign(n, -1);
  acc = 0;
  for (TileInfo& ti : P.tiles) {
    ti.lut_base_lo = (uint32_t)acc;
    ti.lut_base_hi = (uint32_t)(acc >> 32);
    for (int m = 0; m < ti.count; ++m) {
      const int idx = P.tile_neuron[ti.first + m];
      P.lut_off[idx] = acc;
      P.tile_pos[idx] = ti.first + m;
      acc += (uint64_t)P.lut_cap[idx];
    }
  }
  for (const Group& G : P.groups)
    if (G.wide_wb)
      for (int k = G.neuron_begin; k < G.neuron_end; ++k) {
        const int idx = P.group_neurons[k];
        P.lut_off[idx] = acc;
        acc += (uint64_t)P.lut_cap[idx];
      }
  P.lut_total = acc;
  for (WorkItem& w : P.items) w.t = P.tiles[w.tile];
  if (persistent) {
    // Longest processing time first: cost ~ words x neurons x thresholds
    // plus the mask-table copy.
    auto cost = [&](const WorkItem& w) {
      const TileInfo& t = P.tiles[w.tile];
      return (double)w.count * (double)t.count * (double)((1 << t.o) + 1) + 4.0 * (double)t.lut_total;
    };
    std::stable_sort(P.items.begin(), P.items.end(),
                     [&](const WorkItem& x, const WorkItem& y) { return cost(x) > cost(y); });
  }
  build_large_list(P);
}

// ------------------------------------------------------ device workspace
struct Layout {
  size_t desc, lut_off, lut_cap, tiles, tile_neuron, tile_lds, tile_pos, items, group_neurons, large, sup_lists;
  size_t upload_bytes;
  size_t params, slots, queue, found, sup_list, sup_count, lut;
  size_t total;
};

Layout layout_of(const PlanHost& P) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.desc = take(sizeof(tt_neuron) * P.desc.size());
  L.lut_off = take(sizeof(uint64_t) * P.lut_off.size());
  L.lut_cap = take(sizeof(int32_t) * P.lut_cap.size());
  L.tiles = take(sizeof(TileInfo) * P.tiles.size());
  L.tile_neuron = take(sizeof(int32_t) * P.tile_neuron.size());
  L.tile_lds = take(sizeof(int32_t) * P.tile_lds.size());
  L.tile_pos = take(sizeof(int32_t) * P.tile_pos.size());
  L.items = take(sizeof(WorkItem) * P.items.size());
  L.group_neurons = take(sizeof(int32_t) * P.group_neurons.size());
  L.large = take(sizeof(int32_t) * P.large.size());
  L.sup_lists = take(sizeof(int32_t) * P.sup_lists.size());
  L.upload_bytes = o;
  L.params = take(sizeof(NeuronParams) * P.desc.size());
  L.slots = take(sizeof(LdsSlot) * P.tile_neuron.size());
  L.queue = take(sizeof(uint32_t) * 4);
  L.found = take(sizeof(uint32_t) * P.desc.size());
  L.sup_list = take(sizeof(int32_t) * (size_t)P.n);  // neurons still pending a support check
  L.sup_count = take(sizeof(uint32_t) * 4);
  L.lut = take(sizeof(uint64_t) * P.lut_total);
  L.total = o;
  return L;
}

std::vector<uint8_t>* make_upload(const PlanHost& P, const Layout& L) {
  auto* blob = new std::vector<uint8_t>(L.upload_bytes, 0);
  auto put = [&](size_t at, const void* src, size_t bytes) {
    if (bytes) std::memcpy(blob->data() + at, src, bytes);
  };
  put(L.desc, P.desc.data(), sizeof(tt_neuron) * P.desc.size());
  put(L.lut_off, P.lut_off.data(), sizeof(uint64_t) * P.lut_off.size());
  put(L.lut_cap, P.lut_cap.data(), sizeof(int32_t) * P.lut_cap.size());
  put(L.tiles, P.tiles.data(), sizeof(TileInfo) * P.tiles.size());
  put(L.tile_neuron, P.tile_neuron.data(), sizeof(int32_t) * P.tile_neuron.size());
  put(L.tile_lds, P.tile_lds.data(), sizeof(int32_t) * P.tile_lds.size());
  put(L.tile_pos, P.tile_pos.data(), sizeof(int32_t) * P.tile_pos.size());
  put(L.items, P.items.data(), sizeof(WorkItem) * P.items.size());
  put(L.group_neurons, P.group_neurons.data(), sizeof(int32_t) * P.group_neurons.size());
  put(L.large, P.large.data(), sizeof(int32_t) * P.large.size());
  put(L.sup_lists, P.sup_lists.data(), sizeof(int32_t) * P.sup_lists.size());
  return blob;
}

void free_blob(void* p) { delete static_cast<std::vector<uint8_t>*>(p); }

// Stream-ordered upload of a host blob; the blob is freed by a host callback
// once the copy has executed.
int upload_async(void* dst, std::vector<uint8_t>* blob, hipStream_t s) {
  if (blob->empty()) {
    delete blob;
    return TT_OK;
  }
  hipError_t e = hipMemcpyAsync(dst, blob->data(), blob->size(), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    delete blob;
    g_last_hip = (int)e;
    return TT_EHIP;
  }
  e = hipLaunchHostFunc(s, free_blob, blob);
  if (e != hipSuccess) {
    // The copy is already queued: wait for it before releasing the blob.
    (void)hipStreamSynchronize(s);
    delete blob;
    g_last_hip = (int)e;
    return TT_EHIP;
  }
  return TT_OK;
}

EnumArgs enum_args(const PlanHost& P, const Layout& L, uint8_t* ws, uint64_t* tables) {
  EnumArgs a{};
  a.desc = reinterpret_cast<const tt_neuron*>(ws + L.desc);
  a.lut_off = reinterpret_cast<const uint64_t*>(ws + L.lut_off);
  a.lut_cap = reinterpret_cast<const int32_t*>(ws + L.lut_cap);
  a.params = reinterpret_cast<NeuronParams*>(ws + L.params);
  a.lut = reinterpret_cast<uint64_t*>(ws + L.lut);
  a.tiles = reinterpret_cast<const TileInfo*>(ws + L.tiles);
  a.tile_neuron = reinterpret_cast<const int32_t*>(ws + L.tile_neuron);
  a.tile_lds = reinterpret_cast<const int32_t*>(ws + L.tile_lds);
  a.tile_pos = reinterpret_cast<const int32_t*>(ws + L.tile_pos);
  a.slots = reinterpret_cast<LdsSlot*>(ws + L.slots);
  a.tile_lut_max = 1;
  for (const TileInfo& ti : P.tiles) a.tile_lut_max = std::max(a.tile_lut_max, (int32_t)ti.lut_total);
  a.items = reinterpret_cast<const WorkItem*>(ws + L.items);
  a.queue = reinterpret_cast<uint32_t*>(ws + L.queue);
  a.prep_waves = 1;
  a.tables = tables;
  (void)P;
  return a;
}

int grid_for(const PlanHost& P, int cus) {
  const long g = (long)P.tune.blocks_per_cu * (long)cus;
  return (int)std::max<long>(1, std::min<long>(g, (long)P.items.size()));
}

// Enqueue support and/or histogram of the plan's neurons over `tables`
// (see tt_support.hip): the histogram by one counting pass over the words,
// the support by probes, a device-side list of the neurons still pending and
// work units over their unknown digits.
int enqueue_support(const PlanHost& P, const Layout& L, uint8_t* ws, const uint64_t* tables, uint8_t* support,
                    uint32_t* hist, hipStream_t s, bool own_tables = false, bool small_done = false) {
  if (P.n == 0) return TT_OK;
  if (own_tables && support) {
    // the tables are the enumeration of these descriptors: the support
    // follows from the parameters, no table read (neurons with sums below
    // 512 values one wave each, unless the enumeration's prep pass already
    // decided them; the others one block each)
    const tt_neuron* d = reinterpret_cast<const tt_neuron*>(ws + L.desc);
    const int32_t* lists = reinterpret_cast<const int32_t*>(ws + L.sup_lists);
    const int ns = (int)P.sup_small;
    if (!small_done) TT_HIP(launch_support_params_small(d, lists, ns, support, s));
    TT_HIP(launch_support_params(d, lists + ns, P.n - ns, support, s));
    if (!hist) return TT_OK;
    support = nullptr;  // the histogram below is counted from the tables
  }
  SupportArgs sa{};
  sa.desc = reinterpret_cast<const tt_neuron*>(ws + L.desc);
  sa.tables = tables;
  sa.found = reinterpret_cast<uint32_t*>(ws + L.found);
  sa.hist = hist;
  sa.support = support;
  sa.n = P.n;
  sa.n_large = (int32_t)P.large.size();
  sa.large = reinterpret_cast<const int32_t*>(ws + L.large);
  int cus = 0;
  TT_TRY(device_info(&cus));
  // Tables of at most kSmallTableWords words per plane: one thread per
  // neuron.  Larger ones: work units per neuron, about four (histogram:
  // every large neuron) or eight (support: only the neurons still pending)
  // per resident wave in all.
  const long nl = std::max<long>(1, sa.n_large);
  auto units = [&](long per_wave, long cap) {
    const long target = per_wave * 32L * cus;
    return (int)std::max<long>(1, std::min<long>(cap, (target + nl - 1) / nl));
  };
  if (hist) TT_HIP(launch_fill_u32(hist, (size_t)P.n * 8, 0u, s));
  TT_HIP(launch_small_tables(sa, s));
  if (hist) TT_HIP(launch_hist_tables(sa, (int)std::min<long>(units(4, 64), P.max_chunks), s));
  if (support && sa.n_large > 0) {
    const int U = (int)std::min<long>(units(8, 128), P.max_items);
    TT_HIP(launch_fill_u32(sa.found, (size_t)P.n, 0u, s));
    TT_HIP(launch_support_tasks(sa, U, reinterpret_cast<int32_t*>(ws + L.sup_list),
                                reinterpret_cast<uint32_t*>(ws + L.sup_count), s));
    TT_HIP(launch_support_finish(sa, s));
  }
  return TT_OK;
}

// Enqueue the whole enumeration.  With hist != NULL the enumeration kernels
// also form the histogram (tile kernel: each work item adds its share; wide
// groups: their counts kernel).  With small_support != NULL the prep pass
// also decides the support of the neurons whose sums span fewer than 512
// values.
int enqueue_plan(const PlanHost& P, const Layout& L, uint8_t* ws, uint64_t* tables, uint32_t* hist,
                 int cus, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                 uint8_t* small_support = nullptr) {
  if (P.n == 0) return TT_OK;
  EnumArgs a = enum_args(P, L, ws, tables);
  a.hist = hist;
  a.support = small_support;
  // Prep waves per neuron: each wave's dependent chain is the kernel's time
  // when the neurons are few, so the mask-table chunks and the support get
  // waves of their own, up to one round of resident waves (8 per SIMD).
  {
    const long round = 32L * (long)std::max(cus, 1);
    const long fit = round / std::max<long>(P.n, 1);
    a.prep_waves = (int)std::max<long>(1, std::min<long>(fit, 1 + P.lut_chunks));
  }
  const bool persistent = (P.flags & TT_PLAN_PERSISTENT) != 0;
  const int32_t* gn = reinterpret_cast<const int32_t*>(ws + L.group_neurons);
  auto launch_wide = [&](const Group& G) {
    a.wide_list = gn + G.neuron_begin;
    a.wide_count = G.neuron_end - G.neuron_begin;
    a.wide_wb = G.wide_wb;
    a.wide_lds = G.wide_lds;
    a.wide_upw = G.wide_upw;
    return launch_enum_wide(a, G.o, P.tune.waves, P.tune.nontemporal, s);
  };
  if (persistent) {
    a.prep_list = nullptr;
    a.prep_count = P.n;
    TT_HIP(launch_prep(a, s));
    if (ev0) TT_HIP(hipEventRecord(ev0, s));
    for (const Group& G : P.groups)
      if (G.wide_wb) TT_HIP(launch_wide(G));
    a.persistent = 1;
    a.item_base = 0;
    a.n_items = (int)P.items.size();
    if (a.n_items > 0)
      TT_HIP(launch_enum(a, grid_for(P, cus), P.tune.waves, P.tune.nontemporal, P.tune.tile_neurons, s));
    if (ev1) TT_HIP(hipEventRecord(ev1, s));
  } else {
    if (ev0) TT_HIP(hipEventRecord(ev0, s));
    for (const Group& G : P.groups) {
      a.prep_list = gn + G.neuron_begin;
      a.prep_count = G.neuron_end - G.neuron_begin;
      a.queue = nullptr;
      TT_HIP(launch_prep(a, s));
      if (G.wide_wb) {
        TT_HIP(launch_wide(G));
        continue;
      }
      a.persistent = 0;
      a.item_base = G.item_begin;
      a.n_items = G.item_end;
      TT_HIP(launch_enum(a, G.item_end - G.item_begin, P.tune.waves, P.tune.nontemporal, P.tune.tile_neurons, s));
    }
    if (ev1) TT_HIP(hipEventRecord(ev1, s));
  }
  return TT_OK;
}

// Validate the arguments of a one-shot enumeration and build its plan
// (groups of (F, b, o), each enumerated by its own launches).
int plan_oneshot(const tt_neuron* h_desc, int n, const uint64_t* d_tables, uint64_t total_words, PlanHost* P) {
  TT_TRY(validate_all(h_desc, n));
  if (n == 0) return TT_OK;
  if (!d_tables) return TT_EINVAL;
  TT_TRY(validate_ranges(h_desc, n, total_words));
  P->n = n;
  P->total_words = total_words;
  P->tune = default_tune();
  P->flags = 0;
  P->desc.assign(h_desc, h_desc + n);
  build_plan(*P, false);
  return TT_OK;
}

// Fixed workspace of tt_enumerate_noalloc, for callers that cannot allocate
// device memory.  Every device the library runs on holds its own copy until
// the process ends.  In host code `scratch` names a host-side stand-in, so
// its device address is taken once per device with hipGetSymbolAddress and
// only that address is handed to kernels and copies.
constexpr size_t kNoallocScratchBytes = (size_t)TT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kNoallocScratchBytes];

std::mutex g_scratch_mu;
std::map<int, uint8_t*> g_scratch_ptr;

int noalloc_scratch(uint8_t** ptr) {
  int dev = 0;
  TT_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    TT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return TT_EHIP;
    it = g_scratch_ptr.emplace(dev, static_cast<uint8_t*>(p)).first;
  }
  *ptr = it->second;
  return TT_OK;
}

}  // namespace

// ====================================================================== ABI
struct tt_plan {
  PlanHost host;
  Layout layout{};
  uint8_t* ws = nullptr;
  int cus = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t* cap_tables = nullptr;
  uint32_t* cap_hist = nullptr;
  // the captured whole step (tt_plan_step)
  hipGraph_t step_graph = nullptr;
  hipGraphExec_t step_exec = nullptr;
  uint64_t* step_tables = nullptr;
  uint32_t* step_hist = nullptr;
  uint8_t* step_support = nullptr;
  static constexpr int kTimingRing = 256;
  std::vector<hipEvent_t> ev;  // 2 * kTimingRing events with TT_PLAN_TIMING
  long launches = 0, read = 0;
};

// ----------------------------------------------------------------- CNF
struct tt_cnf {
  int n_inst = 0, n_clauses = 0, max_vars = 0;
  uint8_t* ws = nullptr;
  tt::CnfArgs args{};
};

struct tt_gd {
  uint8_t* ws = nullptr;
  tt::GdArgs args{};
  std::vector<int32_t> pi_vars;  // variable of each logit column
  hipModule_t mod = nullptr;      // the circuit's compiled kernel (NULL: none)
  hipFunction_t fn = nullptr;
  int kernel = TT_GD_INTERPRETED;  // the kernel tt_gd_run launches
};

// ------------------------------------------------------------- networks
struct tt_lutnet {
  int n = 0, n_inputs = 0, depth = 0;
  long stride = 0;      // > 0: the single-launch form
  uint8_t* ws = nullptr;
  bool ws_async = false;  // allocated in stream order (freed the same way)
  tt::NetArgs na{};
  tt::LutnetArgs la{};
  std::vector<int> level_begin;
  const int32_t* order = nullptr;  // device, per-level form
};

namespace {

// Validate a network, group it by level and build its workspace (records,
// interleaved tables and input masks for the single-launch form; descriptors,
// fan-in and level order for the per-level form).  check_only: stop after
// the argument checks.
int lutnet_setup(const tt_neuron* h_desc, int n, const int32_t* h_fanin, int n_inputs, const uint64_t* d_tables,
                 uint64_t total_words, hipStream_t s, bool async_ws, tt_lutnet* L, bool check_only = false) {
  TT_TRY(validate_all(h_desc, n));
  if (n_inputs < 0 || (n > 0 && !h_fanin)) return TT_EINVAL;
  // fan-in: signals below n_inputs + i (topological order); levels from it
  std::vector<int32_t> level(n, 0);
  int depth = 0;
  for (int i = 0; i < n; ++i) {
    int lv = 0;
    for (int j = 0; j < h_desc[i].F; ++j) {
      const int32_t sig = h_fanin[8 * (size_t)i + j];
      if (sig < 0 || (int64_t)sig >= (int64_t)n_inputs + i) return TT_EINVAL;
      if (sig >= n_inputs) lv = std::max(lv, level[sig - n_inputs] + 1);
    }
    level[i] = lv;
    depth = std::max(depth, lv + 1);
  }
  L->n = n;
  L->n_inputs = n_inputs;
  L->depth = depth;
  if (n == 0 || check_only) return TT_OK;
  if (!d_tables) return TT_EINVAL;
  TT_TRY(validate_ranges(h_desc, n, total_words));
  TT_TRY(device_info(nullptr));
  // neurons grouped by level
  std::vector<int32_t> order;
  L->level_begin.assign(depth + 1, 0);
  order.reserve(n);
  for (int lv = 0; lv < depth; ++lv) {
    L->level_begin[lv] = (int)order.size();
    for (int i = 0; i < n; ++i)
      if (level[i] == lv) order.push_back(i);
  }
  L->level_begin[depth] = (int)order.size();
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const long stride = tt::lutnet_fused_stride(n_inputs, n);
  L->stride = stride;
  std::vector<uint8_t>* blob = nullptr;
  size_t off_rec = 0, off_lvb = 0, off_inm = 0, off_rep = 0, off_il = 0;
  size_t off_desc = 0, off_fan = 0, off_ord = 0;
  int fmax = 1, omax = 1;
  bool need_mask = false;
  if (stride > 0) {
    for (int i = 0; i < n; ++i) {
      fmax = std::max(fmax, (int)h_desc[i].F);
      omax = std::max(omax, (int)h_desc[i].o);
    }
    const int G = tt::net_group(omax);
    uint64_t il_dwords = 0;
    for (int i = 0; i < n; ++i) {
      const int Fb = h_desc[i].F * h_desc[i].b;
      il_dwords += (uint64_t)G * (Fb > 5 ? 1ull << (Fb - 5) : 1ull);
    }
    off_rec = take(sizeof(tt::NetRec) * n);
    off_lvb = take(sizeof(int32_t) * (depth + 1));
    off_inm = take((size_t)n_inputs);
    off_rep = take(sizeof(tt::RepackItem) * n);
    const size_t blob_bytes = o;
    off_il = take(4 * il_dwords);
    blob = new std::vector<uint8_t>(blob_bytes, 0);
    auto* rec = reinterpret_cast<tt::NetRec*>(blob->data() + off_rec);
    auto* rep = reinterpret_cast<tt::RepackItem*>(blob->data() + off_rep);
    uint64_t at = 0;
    for (int k = 0; k < n; ++k) {
      const int i = order[k];
      const tt_neuron& d = h_desc[i];
      const int Fb = d.F * d.b;
      const uint32_t groups = Fb > 5 ? 1u << (Fb - 5) : 1u;
      tt::NetRec& R = rec[k];
      R.tab = at;
      R.out = (uint32_t)(n_inputs + i);
      R.mask = (1u << d.b) - 1u;
      R.b = d.b;
      for (int j = 0; j < 8; ++j) R.sig[j] = (uint32_t)(j < d.F ? h_fanin[8 * (size_t)i + j] : n_inputs + n);
      rep[k] = tt::RepackItem{d.word_off, at, (uint32_t)words_of(d.F, d.b), d.o, groups, 0u};
      at += (uint64_t)G * groups;
    }
    std::memcpy(blob->data() + off_lvb, L->level_begin.data(), sizeof(int32_t) * (depth + 1));
    // An input whose readers all take b digits is staged as its low b bits;
    // then no reader has to mask unless some input has readers of different
    // b, or some neuron's o exceeds a reader's b.
    std::vector<int> in_b(n_inputs, 0);  // 0: no reader yet, -1: readers differ
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < h_desc[i].F; ++j) {
        const int32_t sg = h_fanin[8 * (size_t)i + j];
        const int b = h_desc[i].b;
        if (sg < n_inputs)
          in_b[sg] = in_b[sg] == 0 || in_b[sg] == b ? b : -1;
        else if (h_desc[sg - n_inputs].o > b)
          need_mask = true;
      }
    uint8_t* inm = blob->data() + off_inm;
    for (int sg = 0; sg < n_inputs; ++sg) {
      need_mask = need_mask || in_b[sg] < 0;
      inm[sg] = in_b[sg] > 0 ? (uint8_t)((1u << in_b[sg]) - 1u) : (uint8_t)0xFF;
    }
  } else {
    off_desc = take(sizeof(tt_neuron) * n);
    off_fan = take(sizeof(int32_t) * 8 * (size_t)n);
    off_ord = take(sizeof(int32_t) * n);
    blob = new std::vector<uint8_t>(o, 0);
    std::memcpy(blob->data() + off_desc, h_desc, sizeof(tt_neuron) * n);
    std::memcpy(blob->data() + off_fan, h_fanin, sizeof(int32_t) * 8 * (size_t)n);
    std::memcpy(blob->data() + off_ord, order.data(), sizeof(int32_t) * n);
  }
  hipError_t e = async_ws ? hipMallocAsync((void**)&L->ws, o, s) : hipMalloc((void**)&L->ws, o);
  if (e != hipSuccess) {
    delete blob;
    L->ws = nullptr;
    g_last_hip = (int)e;
    return TT_ENOMEM;
  }
  L->ws_async = async_ws;
  TT_TRY(upload_async(L->ws, blob, s));
  if (stride > 0) {
    tt::NetArgs& na = L->na;
    na.rec = reinterpret_cast<const tt::NetRec*>(L->ws + off_rec);
    na.level_begin = reinterpret_cast<const int32_t*>(L->ws + off_lvb);
    na.depth = depth;
    na.n_inputs = n_inputs;
    na.n = n;
    na.stride = (int32_t)stride;
    na.fmax = fmax;
    na.omax = omax;
    na.mask = need_mask ? 1 : 0;
    na.in_mask = L->ws + off_inm;
    na.tables = reinterpret_cast<const uint32_t*>(L->ws + off_il);
    TT_HIP(tt::launch_lutnet_repack(reinterpret_cast<const tt::RepackItem*>(L->ws + off_rep), n,
                                    tt::net_group(omax), d_tables, reinterpret_cast<uint32_t*>(L->ws + off_il), s));
  } else {
    tt::LutnetArgs& la = L->la;
    la.desc = reinterpret_cast<const tt_neuron*>(L->ws + off_desc);
    la.fanin = reinterpret_cast<const int32_t*>(L->ws + off_fan);
    la.n_inputs = n_inputs;
    la.n = n;
    la.tables = d_tables;
    L->order = reinterpret_cast<const int32_t*>(L->ws + off_ord);
  }
  return TT_OK;
}

int lutnet_enqueue(const tt_lutnet& L, const uint8_t* d_inputs, int batch, uint8_t* d_out, hipStream_t s) {
  if (L.stride > 0) {
    tt::NetArgs na = L.na;
    na.batch = batch;
    na.inputs = d_inputs;
    na.out = d_out;
    na.sample = 0;
    TT_HIP(tt::launch_lutnet_fused(na, tt::NetSample{}, s));
    return TT_OK;
  }
  tt::LutnetArgs la = L.la;
  la.batch = batch;
  la.inputs = d_inputs;
  la.out = d_out;
  for (int lv = 0; lv < L.depth; ++lv) {
    la.level = L.order + L.level_begin[lv];
    la.count = L.level_begin[lv + 1] - L.level_begin[lv];
    TT_HIP(tt::launch_lutnet_level(la, s));
  }
  return TT_OK;
}

// Free the workspace (in stream order when it was allocated that way).
int lutnet_release(tt_lutnet* L, hipStream_t s) {
  if (!L->ws) return TT_OK;
  const hipError_t e = L->ws_async ? hipFreeAsync(L->ws, s) : hipFree(L->ws);
  L->ws = nullptr;
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    return TT_EHIP;
  }
  return TT_OK;
}

}  // namespace

extern "C" {

const char* tt_strerror(int status) {
  switch (status) {
    case TT_OK: return "success";
    case TT_EINVAL: return "invalid argument";
    case TT_ERANGE: return "value out of range";
    case TT_EHIP: return "HIP runtime error";
    case TT_ENOMEM: return "out of memory";
    case TT_ENOTSUP: return "device is not gfx950";
    case TT_ESCRATCH: return "input needs more workspace than the fixed scratch of tt_enumerate_noalloc";
    default: return "unknown status";
  }
}

int tt_last_hip_error(void) { return g_last_hip; }

int tt_version(void) { return (1 << 16) | 0; }

int tt_device_check(void) { return device_info(nullptr); }

uint64_t tt_words_per_plane(int F, int b) {
  if (F < 1 || F > TT_MAX_F || b < 1 || b > TT_MAX_B || F * b > TT_MAX_FB) return 0;
  return words_of(F, b);
}

int tt_validate(const tt_neuron* h_desc, int n) { return validate_all(h_desc, n); }

int tt_layout(tt_neuron* h_desc, int n, uint64_t* h_total_words) {
  if (!h_total_words) return TT_EINVAL;
  TT_TRY(validate_all(h_desc, n));
  uint64_t acc = 0;
  for (int i = 0; i < n; ++i) {
    h_desc[i].word_off = acc;
    acc += (uint64_t)h_desc[i].o * words_of(h_desc[i].F, h_desc[i].b);
  }
  *h_total_words = acc;
  return TT_OK;
}

int tt_enumerate(const tt_neuron* h_desc, int n, uint64_t* d_tables, uint64_t total_words,
                 uint32_t* d_hist, void* stream) {
  PlanHost P;
  TT_TRY(plan_oneshot(h_desc, n, d_tables, total_words, &P));
  if (n == 0) return TT_OK;
  int cus = 0;
  TT_TRY(device_info(&cus));
  hipStream_t s = (hipStream_t)stream;
  const Layout L = layout_of(P);
  uint8_t* ws = nullptr;
  hipError_t e = hipMallocAsync((void**)&ws, L.total, s);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    return TT_ENOMEM;
  }
  int st = upload_async(ws, make_upload(P, L), s);
  if (st == TT_OK) st = enqueue_plan(P, L, ws, d_tables, d_hist, cus, s);
  e = hipFreeAsync(ws, s);
  if (st == TT_OK && e != hipSuccess) {
    g_last_hip = (int)e;
    st = TT_EHIP;
  }
  return st;
}

int tt_enumerate_noalloc(const tt_neuron* h_desc, int n, uint64_t* d_tables, uint64_t total_words,
                         uint32_t* d_hist, void* stream) {
  PlanHost P;
  TT_TRY(plan_oneshot(h_desc, n, d_tables, total_words, &P));
  if (n == 0) return TT_OK;
  const Layout L = layout_of(P);
  if (L.total > kNoallocScratchBytes) return TT_ESCRATCH;
  int cus = 0;
  TT_TRY(device_info(&cus));
  uint8_t* ws = nullptr;
  TT_TRY(noalloc_scratch(&ws));
  hipStream_t s = (hipStream_t)stream;
  const int st = upload_async(ws, make_upload(P, L), s);
  return st == TT_OK ? enqueue_plan(P, L, ws, d_tables, d_hist, cus, s) : st;
}

int tt_plan_create(const tt_neuron* h_desc, int n, uint64_t total_words, const tt_tune* tune,
                   unsigned flags, tt_plan** plan) {
  if (!plan) return TT_EINVAL;
  *plan = nullptr;
  TT_TRY(validate_all(h_desc, n));
  TT_TRY(validate_ranges(h_desc, n, total_words));
  const tt_tune t = tune ? *tune : default_tune();
  TT_TRY(check_tune(t));
  int cus = 0;
  TT_TRY(device_info(&cus));
  tt_plan* p = new (std::nothrow) tt_plan();
  if (!p) return TT_ENOMEM;
  p->host.n = n;
  p->host.total_words = total_words;
  p->host.tune = t;
  p->host.flags = flags;
  p->host.desc.assign(h_desc, h_desc + n);
  build_plan(p->host, (flags & TT_PLAN_PERSISTENT) != 0);
  p->layout = layout_of(p->host);
  p->cus = cus;
  hipError_t e = hipMalloc((void**)&p->ws, std::max<size_t>(p->layout.total, kAlign));
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    delete p;
    return TT_ENOMEM;
  }
  std::vector<uint8_t>* blob = make_upload(p->host, p->layout);
  e = blob->empty() ? hipSuccess : hipMemcpy(p->ws, blob->data(), blob->size(), hipMemcpyHostToDevice);
  delete blob;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess && (flags & TT_PLAN_TIMING) && !(flags & TT_PLAN_GRAPH)) {
    // timing only: no system-scope fence (cache writeback and invalidate)
    // when an event completes, so the events barely disturb the step
    p->ev.assign(2 * tt_plan::kTimingRing, nullptr);
    for (auto& x : p->ev)
      if (e == hipSuccess) e = hipEventCreateWithFlags(&x, hipEventDisableSystemFence);
  }
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    (void)hipFree(p->ws);
    delete p;
    return TT_EHIP;
  }
  *plan = p;
  return TT_OK;
}

int tt_plan_launch(tt_plan* p, uint64_t* d_tables, uint32_t* d_hist, void* stream) {
  if (!p) return TT_EINVAL;
  if (p->host.n == 0) return TT_OK;
  if (!d_tables) return TT_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (!(p->host.flags & TT_PLAN_GRAPH)) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!p->ev.empty()) {
      const int slot = (int)(p->launches % tt_plan::kTimingRing);
      e0 = p->ev[2 * slot];
      e1 = p->ev[2 * slot + 1];
    }
    const int st = enqueue_plan(p->host, p->layout, p->ws, d_tables, d_hist, p->cus, s, e0, e1);
    if (st == TT_OK && e0) ++p->launches;
    return st;
  }
  if (!p->exec || p->cap_tables != d_tables || p->cap_hist != d_hist) {
    if (p->exec) {
      TT_HIP(hipGraphExecDestroy(p->exec));
      p->exec = nullptr;
    }
    if (p->graph) {
      TT_HIP(hipGraphDestroy(p->graph));
      p->graph = nullptr;
    }
    TT_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    const int st = enqueue_plan(p->host, p->layout, p->ws, d_tables, d_hist, p->cus, p->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (st != TT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    TT_HIP(e);
    p->graph = g;
    TT_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    p->cap_tables = d_tables;
    p->cap_hist = d_hist;
  }
  TT_HIP(hipGraphLaunch(p->exec, s));
  return TT_OK;
}

int tt_plan_step(tt_plan* p, uint64_t* d_tables, uint32_t* d_hist, uint8_t* d_support, void* stream) {
  if (!p) return TT_EINVAL;
  if (p->host.n == 0) return TT_OK;
  if (!d_tables) return TT_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  auto enqueue = [&](hipStream_t q, hipEvent_t e0, hipEvent_t e1) {
    int st = enqueue_plan(p->host, p->layout, p->ws, d_tables, d_hist, p->cus, q, e0, e1, d_support);
    if (st == TT_OK && d_support)
      st = enqueue_support(p->host, p->layout, p->ws, d_tables, d_support, nullptr, q, true, true);
    return st;
  };
  if (!(p->host.flags & TT_PLAN_GRAPH)) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!p->ev.empty()) {
      const int slot = (int)(p->launches % tt_plan::kTimingRing);
      e0 = p->ev[2 * slot];
      e1 = p->ev[2 * slot + 1];
    }
    const int st = enqueue(s, e0, e1);
    if (st == TT_OK && e0) ++p->launches;
    return st;
  }
  if (!p->step_exec || p->step_tables != d_tables || p->step_hist != d_hist || p->step_support != d_support) {
    if (p->step_exec) {
      TT_HIP(hipGraphExecDestroy(p->step_exec));
      p->step_exec = nullptr;
    }
    if (p->step_graph) {
      TT_HIP(hipGraphDestroy(p->step_graph));
      p->step_graph = nullptr;
    }
    TT_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    const int st = enqueue(p->cap_stream, nullptr, nullptr);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (st != TT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    TT_HIP(e);
    p->step_graph = g;
    TT_HIP(hipGraphInstantiate(&p->step_exec, p->step_graph, nullptr, nullptr, 0));
    p->step_tables = d_tables;
    p->step_hist = d_hist;
    p->step_support = d_support;
  }
  TT_HIP(hipGraphLaunch(p->step_exec, s));
  return TT_OK;
}

int tt_plan_destroy(tt_plan* p) {
  if (!p) return TT_OK;
  int st = TT_OK;
  if (hipDeviceSynchronize() != hipSuccess) st = TT_EHIP;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->step_exec) (void)hipGraphExecDestroy(p->step_exec);
  if (p->step_graph) (void)hipGraphDestroy(p->step_graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (auto x : p->ev)
    if (x) (void)hipEventDestroy(x);
  if (p->ws) (void)hipFree(p->ws);
  delete p;
  return st;
}

int tt_plan_kernel_times(tt_plan* p, float* h_ms, int max_count, int* count) {
  if (!p || !count || (max_count > 0 && !h_ms)) return TT_EINVAL;
  *count = 0;
  if (p->ev.empty()) return TT_EINVAL;
  long first = std::max(p->read, p->launches - (long)tt_plan::kTimingRing);
  int c = 0;
  for (long i = first; i < p->launches && c < max_count; ++i, ++c) {
    const int slot = (int)(i % tt_plan::kTimingRing);
    TT_HIP(hipEventSynchronize(p->ev[2 * slot + 1]));
    float ms = 0.f;
    TT_HIP(hipEventElapsedTime(&ms, p->ev[2 * slot], p->ev[2 * slot + 1]));
    h_ms[c] = ms;
  }
  p->read = first + c;
  *count = c;
  return TT_OK;
}

int tt_plan_wide_neurons(const tt_plan* p, int* n_wide) {
  if (!p || !n_wide) return TT_EINVAL;
  int c = 0;
  for (const Group& G : p->host.groups)
    if (G.wide_wb) c += G.neuron_end - G.neuron_begin;
  *n_wide = c;
  return TT_OK;
}

int tt_plan_info(const tt_plan* p, tt_tune* tune, int* n_items, int* n_groups, int* grid) {
  if (!p) return TT_EINVAL;
  if (tune) *tune = p->host.tune;
  if (n_items) *n_items = (int)p->host.items.size();
  if (n_groups) *n_groups = (int)p->host.groups.size();
  if (grid) *grid = (p->host.flags & TT_PLAN_PERSISTENT) ? grid_for(p->host, p->cus) : -1;
  return TT_OK;
}

// ------------------------------------------------------------ tt_support
int tt_support(const tt_neuron* h_desc, int n, const uint64_t* d_tables, uint64_t total_words,
               uint8_t* d_support, uint32_t* d_hist, void* stream) {
  TT_TRY(validate_all(h_desc, n));
  if (n == 0) return TT_OK;
  if (!d_tables || (!d_support && !d_hist)) return TT_EINVAL;
  TT_TRY(validate_ranges(h_desc, n, total_words));
  TT_TRY(device_info(nullptr));
  hipStream_t s = (hipStream_t)stream;
  PlanHost P;
  P.n = n;
  P.desc.assign(h_desc, h_desc + n);
  build_large_list(P);
  const Layout L = layout_of(P);
  uint8_t* ws = nullptr;
  hipError_t e = hipMallocAsync((void**)&ws, L.total, s);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    return TT_ENOMEM;
  }
  int st = upload_async(ws, make_upload(P, L), s);
  if (st == TT_OK) st = enqueue_support(P, L, ws, d_tables, d_support, d_hist, s);
  e = hipFreeAsync(ws, s);
  if (st == TT_OK && e != hipSuccess) {
    g_last_hip = (int)e;
    st = TT_EHIP;
  }
  return st;
}

int tt_plan_support(tt_plan* p, const uint64_t* d_tables, uint8_t* d_support, uint32_t* d_hist, void* stream) {
  if (!p) return TT_EINVAL;
  if (p->host.n == 0) return TT_OK;
  if (!d_tables || (!d_support && !d_hist)) return TT_EINVAL;
  return enqueue_support(p->host, p->layout, p->ws, d_tables, d_support, d_hist, (hipStream_t)stream);
}

int tt_plan_support_enumerated(tt_plan* p, const uint64_t* d_tables, uint8_t* d_support, uint32_t* d_hist,
                               void* stream) {
  if (!p) return TT_EINVAL;
  if (p->host.n == 0) return TT_OK;
  if (!d_tables || (!d_support && !d_hist)) return TT_EINVAL;
  return enqueue_support(p->host, p->layout, p->ws, d_tables, d_support, d_hist, (hipStream_t)stream, true);
}

// --------------------------------------------------------------- tt_pack
// ---------------------------------------------------------- tt_lutnet_*
int tt_lutnet_create(const tt_neuron* h_desc, int n, const int32_t* h_fanin, int n_inputs, const uint64_t* d_tables,
                     uint64_t total_words, void* stream, tt_lutnet** net) {
  if (!net) return TT_EINVAL;
  *net = nullptr;
  tt_lutnet* L = new (std::nothrow) tt_lutnet();
  if (!L) return TT_ENOMEM;
  const int st = lutnet_setup(h_desc, n, h_fanin, n_inputs, d_tables, total_words, (hipStream_t)stream, false, L);
  if (st != TT_OK) {
    if (L->ws) (void)hipStreamSynchronize((hipStream_t)stream);  // queued copies into the workspace
    (void)lutnet_release(L, nullptr);
    delete L;
    return st;
  }
  *net = L;
  return TT_OK;
}

int tt_lutnet_run(const tt_lutnet* net, const uint8_t* d_inputs, int batch, uint8_t* d_out, void* stream) {
  if (!net || batch < 0) return TT_EINVAL;
  if (net->n == 0 || batch == 0) return TT_OK;
  if (!d_inputs || !d_out) return TT_EINVAL;
  return lutnet_enqueue(*net, d_inputs, batch, d_out, (hipStream_t)stream);
}

int tt_lutnet_sample(const tt_lutnet* net, const int32_t* h_target_signal, const uint8_t* h_target_value,
                     int n_targets, uint64_t seed, uint64_t first_draw, int n_draws, uint8_t* d_found_inputs,
                     uint64_t* d_found_draw, int max_found, uint32_t* d_count, void* stream) {
  if (!net || net->n == 0 || n_draws < 0 || max_found < 0 || n_targets < 0 || n_targets > tt::kNetMaxTargets)
    return TT_EINVAL;
  if (n_targets > 0 && (!h_target_signal || !h_target_value)) return TT_EINVAL;
  tt::NetSample smp{};
  for (int t = 0; t < n_targets; ++t) {
    const int32_t sg = h_target_signal[t];
    if (sg < 0 || (int64_t)sg >= (int64_t)net->n_inputs + net->n) return TT_EINVAL;
    smp.tsig[t] = (uint16_t)sg;  // below 1020: the single-launch form's row
    smp.tval[t] = h_target_value[t];
  }
  if (net->stride == 0) return TT_ERANGE;  // signals do not fit a block's LDS rows
  if (n_draws == 0) return TT_OK;
  if (!d_count || (max_found > 0 && (!d_found_inputs || !d_found_draw))) return TT_EINVAL;
  smp.seed = seed;
  smp.first = first_draw;
  smp.found_inputs = d_found_inputs;
  smp.found_draw = d_found_draw;
  smp.count = d_count;
  smp.max_found = max_found;
  smp.n_targets = n_targets;
  tt::NetArgs na = net->na;
  na.batch = n_draws;
  na.inputs = nullptr;
  na.out = nullptr;
  na.sample = 1;
  TT_HIP(tt::launch_lutnet_fused(na, smp, (hipStream_t)stream));
  return TT_OK;
}

int tt_lutnet_destroy(tt_lutnet* net) {
  if (!net) return TT_OK;
  int st = TT_OK;
  if (net->ws && hipDeviceSynchronize() != hipSuccess) st = TT_EHIP;
  const int st2 = lutnet_release(net, nullptr);
  delete net;
  return st != TT_OK ? st : st2;
}

int tt_lutnet_eval(const tt_neuron* h_desc, int n, const int32_t* h_fanin, int n_inputs, const uint64_t* d_tables,
                   uint64_t total_words, const uint8_t* d_inputs, int batch, uint8_t* d_out, void* stream) {
  if (batch < 0 || (n > 0 && batch > 0 && (!d_inputs || !d_out))) return TT_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  tt_lutnet L;
  // with nothing to evaluate only the arguments are checked
  int st = lutnet_setup(h_desc, n, h_fanin, n_inputs, d_tables, total_words, s, true, &L, batch == 0);
  if (st == TT_OK && n > 0 && batch > 0) st = lutnet_enqueue(L, d_inputs, batch, d_out, s);
  const int st2 = lutnet_release(&L, s);
  return st != TT_OK ? st : st2;
}

// ------------------------------------------------------ tt_cnf_transform
int tt_cnf_create(const int32_t* h_lits, const int32_t* h_clause_off, const int32_t* h_inst_off, int n_inst,
                  const int32_t* h_n_vars, void* stream, tt_cnf** out) {
  static_assert(sizeof(tt_cnf_expr) == 640, "tt_cnf_expr layout");
  if (!out) return TT_EINVAL;
  *out = nullptr;
  if (n_inst < 0) return TT_EINVAL;
  if (n_inst > 0 && (!h_inst_off || !h_n_vars)) return TT_EINVAL;
  if (n_inst > 0 && h_inst_off[0] != 0) return TT_EINVAL;
  const int n_clauses = n_inst > 0 ? h_inst_off[n_inst] : 0;
  for (int t = 0; t < n_inst; ++t)
    if (h_inst_off[t + 1] < h_inst_off[t] || h_n_vars[t] < 0 || h_n_vars[t] > 32767) return TT_EINVAL;
  if (n_clauses > 0 && (!h_clause_off || !h_lits)) return TT_EINVAL;
  if (n_clauses > 0 && h_clause_off[0] != 0) return TT_EINVAL;
  for (int c = 0; c < n_clauses; ++c)
    if (h_clause_off[c + 1] <= h_clause_off[c]) return TT_EINVAL;  // no empty clause
  const int n_lits = n_clauses > 0 ? h_clause_off[n_clauses] : 0;
  // literals in range, no clause holding x and -x; per clause the last
  // clause of its instance that uses any of its variables
  std::vector<int32_t> reach(n_clauses, 0), var_off(n_inst, 0);
  int max_vars = 0;
  long acc = 0;
  for (int t = 0; t < n_inst; ++t) {
    const int nv = h_n_vars[t];
    var_off[t] = (int32_t)acc;
    acc += nv + 1;
    if (acc > INT32_MAX) return TT_EINVAL;
    max_vars = std::max(max_vars, nv);
    std::vector<int32_t> last(nv + 1, -1);
    const int c0 = h_inst_off[t], c1 = h_inst_off[t + 1];
    for (int c = c0; c < c1; ++c)
      for (int p = h_clause_off[c]; p < h_clause_off[c + 1]; ++p) {
        const int L = h_lits[p];
        if (L == 0 || std::abs(L) > nv) return TT_EINVAL;
        for (int q = h_clause_off[c]; q < p; ++q)
          if (h_lits[q] == -L) return TT_EINVAL;
        last[std::abs(L)] = c - c0;
      }
    for (int c = c0; c < c1; ++c) {
      int r = 0;
      for (int p = h_clause_off[c]; p < h_clause_off[c + 1]; ++p) r = std::max(r, last[std::abs(h_lits[p])]);
      reach[c] = r;
    }
  }
  // the staged copy holds each clause's distinct literals (a clause is a set:
  // (x x) is the unit clause (x)), in order of first occurrence
  std::vector<int32_t> dlits, dcoff(n_clauses + 1, 0);
  dlits.reserve(n_lits);
  for (int c = 0; c < n_clauses; ++c) {
    const size_t first = dlits.size();
    for (int p = h_clause_off[c]; p < h_clause_off[c + 1]; ++p)
      if (std::find(dlits.begin() + first, dlits.end(), h_lits[p]) == dlits.end()) dlits.push_back(h_lits[p]);
    dcoff[c + 1] = (int32_t)dlits.size();
  }
  const int n_dlits = (int)dlits.size();
  tt_cnf* h = new (std::nothrow) tt_cnf();
  if (!h) return TT_ENOMEM;
  h->n_inst = n_inst;
  h->n_clauses = n_clauses;
  h->max_vars = max_vars;
  if (n_inst == 0) {
    *out = h;
    return TT_OK;
  }
  int st = device_info(nullptr);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t off_lit = take(sizeof(int32_t) * std::max(n_dlits, 1));
  const size_t off_cof = take(sizeof(int32_t) * (n_clauses + 1));
  const size_t off_iof = take(sizeof(int32_t) * (n_inst + 1));
  const size_t off_rch = take(sizeof(int32_t) * std::max(n_clauses, 1));
  const size_t off_vof = take(sizeof(int32_t) * n_inst);
  const size_t off_nv = take(sizeof(int32_t) * n_inst);
  const size_t off_ord = take(sizeof(int32_t) * n_inst);
  // blocks take instances longest first (a stable sort by clause count), so
  // the last waves to finish are short ones
  std::vector<int32_t> order(n_inst);
  for (int t = 0; t < n_inst; ++t) order[t] = t;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return h_inst_off[x + 1] - h_inst_off[x] > h_inst_off[y + 1] - h_inst_off[y];
  });
  if (st == TT_OK) {
    const hipError_t e = hipMalloc((void**)&h->ws, o);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      h->ws = nullptr;
      st = TT_ENOMEM;
    }
  }
  if (st == TT_OK) {
    auto* blob = new std::vector<uint8_t>(o, 0);
    if (n_dlits > 0) std::memcpy(blob->data() + off_lit, dlits.data(), sizeof(int32_t) * n_dlits);
    if (n_clauses > 0) std::memcpy(blob->data() + off_cof, dcoff.data(), sizeof(int32_t) * (n_clauses + 1));
    std::memcpy(blob->data() + off_iof, h_inst_off, sizeof(int32_t) * (n_inst + 1));
    if (n_clauses > 0) std::memcpy(blob->data() + off_rch, reach.data(), sizeof(int32_t) * n_clauses);
    std::memcpy(blob->data() + off_vof, var_off.data(), sizeof(int32_t) * n_inst);
    std::memcpy(blob->data() + off_nv, h_n_vars, sizeof(int32_t) * n_inst);
    std::memcpy(blob->data() + off_ord, order.data(), sizeof(int32_t) * n_inst);
    st = upload_async(h->ws, blob, (hipStream_t)stream);
  }
  if (st != TT_OK) {
    if (h->ws) {
      (void)hipStreamSynchronize((hipStream_t)stream);
      (void)hipFree(h->ws);
    }
    delete h;
    return st;
  }
  tt::CnfArgs& a = h->args;
  a.lits = reinterpret_cast<const int32_t*>(h->ws + off_lit);
  a.clause_off = reinterpret_cast<const int32_t*>(h->ws + off_cof);
  a.inst_off = reinterpret_cast<const int32_t*>(h->ws + off_iof);
  a.clause_reach = reinterpret_cast<const int32_t*>(h->ws + off_rch);
  a.var_off = reinterpret_cast<const int32_t*>(h->ws + off_vof);
  a.n_vars = reinterpret_cast<const int32_t*>(h->ws + off_nv);
  a.order = reinterpret_cast<const int32_t*>(h->ws + off_ord);
  a.n_inst = n_inst;
  for (int t = 0; t < n_inst && n_clauses > 0; ++t) {
    a.stage_clauses = std::max(a.stage_clauses, h_inst_off[t + 1] - h_inst_off[t]);
    a.stage_lits = std::max(a.stage_lits, dcoff[h_inst_off[t + 1]] - dcoff[h_inst_off[t]]);
  }
  *out = h;
  return TT_OK;
}

int tt_cnf_run(const tt_cnf* h, uint8_t* d_var_class, tt_cnf_expr* d_expr, int32_t* d_n_expr, int32_t* d_status,
               void* stream) {
  if (!h) return TT_EINVAL;
  if (h->n_inst == 0) return TT_OK;
  if (!d_var_class || !d_n_expr || !d_status || (h->n_clauses > 0 && !d_expr)) return TT_EINVAL;
  tt::CnfArgs a = h->args;
  a.var_class = d_var_class;
  a.expr = d_expr;
  a.n_expr = d_n_expr;
  a.status = d_status;
  TT_HIP(tt::launch_cnf_transform(a, h->max_vars, (hipStream_t)stream));
  return TT_OK;
}

int tt_cnf_destroy(tt_cnf* h) {
  if (!h) return TT_OK;
  int st = TT_OK;
  if (h->ws) {
    if (hipDeviceSynchronize() != hipSuccess) st = TT_EHIP;
    if (hipFree(h->ws) != hipSuccess) st = TT_EHIP;
  }
  delete h;
  return st;
}

int tt_cnf_transform(const int32_t* h_lits, const int32_t* h_clause_off, const int32_t* h_inst_off, int n_inst,
                     const int32_t* h_n_vars, uint8_t* d_var_class, tt_cnf_expr* d_expr, int32_t* d_n_expr,
                     int32_t* d_status, void* stream) {
  if (n_inst > 0 && (!d_var_class || !d_n_expr || !d_status)) return TT_EINVAL;
  tt_cnf* h = nullptr;
  TT_TRY(tt_cnf_create(h_lits, h_clause_off, h_inst_off, n_inst, h_n_vars, stream, &h));
  int st = tt_cnf_run(h, d_var_class, d_expr, d_n_expr, d_status, stream);
  // the workspace is released once the stream has passed the kernel
  if (h->ws) {
    const hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (st == TT_OK && e != hipSuccess) {
      g_last_hip = (int)e;
      st = TT_EHIP;
    }
    (void)hipFree(h->ws);
    h->ws = nullptr;
  }
  delete h;
  return st;
}

// ------------------------------------------------------------ tt_gd_*
int tt_gd_create(const int32_t* h_lits, const int32_t* h_clause_off, int n_clauses, int n_vars,
                 const tt_cnf_expr* h_expr, int n_expr, const uint8_t* h_var_class, void* stream, tt_gd** out) {
  if (!out) return TT_EINVAL;
  *out = nullptr;
  if (n_clauses < 0 || n_expr < 0 || n_vars < 0 || n_vars > 32767 || !h_var_class) return TT_EINVAL;
  if ((n_clauses > 0 && (!h_lits || !h_clause_off)) || (n_expr > 0 && !h_expr)) return TT_EINVAL;
  for (int i = 0; i < n_expr; ++i) {
    const tt_cnf_expr& e = h_expr[i];
    if (e.kind < TT_CNF_IV || e.kind > TT_CNF_AUX || e.n_vars < 0 || e.n_vars > TT_CNF_MAX_VARS) return TT_EINVAL;
    for (int j = 0; j < e.n_vars; ++j)
      if (e.vars[j] < 1 || e.vars[j] > n_vars) return TT_EINVAL;
    if (e.kind != TT_CNF_AUX && (e.out < 1 || e.out > n_vars)) return TT_EINVAL;
  }
  // slots: primary inputs first, in the order they entered the primary
  // inputs (an expression's variables in ascending index, expressions in the
  // order found: the order in which the transformation appends them), then
  // every other variable the circuit or the clauses use
  std::vector<int32_t> slot(n_vars + 1, -1), pi_vars;
  for (int i = 0; i < n_expr; ++i)
    for (int j = 0; j < h_expr[i].n_vars; ++j) {
      const int x = h_expr[i].vars[j];
      if ((h_var_class[x] & TT_CNF_CLS_PI) && slot[x] < 0) {
        slot[x] = (int32_t)pi_vars.size();
        pi_vars.push_back(x);
      }
    }
  for (int x = 1; x <= n_vars; ++x)  // none, for a completed transformation
    if ((h_var_class[x] & TT_CNF_CLS_PI) && slot[x] < 0) {
      slot[x] = (int32_t)pi_vars.size();
      pi_vars.push_back(x);
    }
  const int n_pi = (int)pi_vars.size();
  int n_vslots = n_pi;
  auto use = [&](int x) {
    if (slot[x] < 0) slot[x] = n_vslots++;
    return slot[x];
  };
  for (int i = 0; i < n_expr; ++i) {
    for (int j = 0; j < h_expr[i].n_vars; ++j) use(h_expr[i].vars[j]);
    if (h_expr[i].kind != TT_CNF_AUX) use(h_expr[i].out);
  }
  std::vector<int32_t> lits;
  for (int c = 0; c < n_clauses; ++c) {
    if (h_clause_off[c + 1] <= h_clause_off[c]) return TT_EINVAL;
    for (int p = h_clause_off[c]; p < h_clause_off[c + 1]; ++p) {
      const int L = h_lits[p], x = std::abs(L);
      if (L == 0 || x > n_vars || !(h_var_class[x] & (TT_CNF_CLS_PI | TT_CNF_CLS_IV | TT_CNF_CLS_PO)))
        return TT_EINVAL;  // every clause variable is classified by a completed transformation
      lits.push_back(use(x) * 2 + (L < 0 ? 1 : 0));
    }
  }
  // Simplify every expression; gates of the intermediate expressions first,
  // then those of the auxiliary outputs.  Temporaries follow the variables.
  struct Prog {
    std::vector<tt::GdGate> g;
    std::vector<int32_t> rng{0};
  } iv, aux;
  std::vector<int32_t> po;
  std::vector<float> cst(n_vslots, 0.f);
  std::vector<tt_gate> form(1 << 15);
  int max_temps = 0;
  for (int i = 0; i < n_expr; ++i) {
    const tt_cnf_expr& e = h_expr[i];
    const int c = (int)(e.table[0] & 1ull);
    if (e.kind == TT_CNF_PO) {  // a constant: fixes its variable, or is a loss term on a primary input
      if (slot[e.out] < n_pi) {
        po.push_back(slot[e.out]);
        po.push_back(c);
      } else {
        cst[slot[e.out]] = (float)c;
      }
      continue;
    }
    int ng = 0, exact = 0;
    int st = tt_simplify(e.table, e.n_vars, (int)form.size(), form.data(), &ng, &exact);
    if (st == TT_ERANGE && ng > (int)form.size()) {
      form.resize(ng);
      st = tt_simplify(e.table, e.n_vars, (int)form.size(), form.data(), &ng, &exact);
    }
    if (st != TT_OK) return st;
    Prog& pr = e.kind == TT_CNF_IV ? iv : aux;
    // an auxiliary output's value goes to one more temporary
    max_temps = std::max(max_temps, e.kind == TT_CNF_IV ? ng - 1 : ng);
    auto opd = [&](int32_t o) {
      const int32_t idx = o & 0xFFFF;
      const int32_t sl = (o & TT_OPD_TEMP) ? tt::kGdTemp | (n_vslots + idx) : slot[e.vars[idx]];
      return sl | ((o & TT_OPD_NEG) ? tt::kGdNeg : 0);
    };
    for (int k = 0; k < ng; ++k) {
      const tt_gate& f = form[k];
      tt::GdGate g{f.op, 0, 0, 0};
      if (f.op == TT_GATE_CONST) {
        g.a = f.a;
      } else {
        g.a = opd(f.a);
        if (f.op != TT_GATE_COPY) g.b = opd(f.b);
      }
      g.dst = f.dst >= 0 ? n_vslots + f.dst : (e.kind == TT_CNF_IV ? slot[e.out] : n_vslots + ng - 1);
      pr.g.push_back(g);
    }
    pr.rng.push_back((int32_t)pr.g.size());
  }
  const int n_slots = n_vslots + max_temps;
  if (n_slots > tt::kGdSlot) return TT_ERANGE;
  for (int32_t& r : aux.rng) r += (int32_t)iv.g.size();
  std::vector<tt::GdGate> gates = iv.g;
  gates.insert(gates.end(), aux.g.begin(), aux.g.end());
  std::vector<int32_t> coff(n_clauses + 1, 0);
  for (int c = 0; c < n_clauses; ++c) coff[c + 1] = h_clause_off[c + 1] - h_clause_off[0];
  TT_TRY(device_info(nullptr));
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t off_gate = take(sizeof(tt::GdGate) * std::max<size_t>(gates.size(), 1));
  const size_t off_iv = take(sizeof(int32_t) * iv.rng.size());
  const size_t off_aux = take(sizeof(int32_t) * aux.rng.size());
  const size_t off_po = take(sizeof(int32_t) * std::max<size_t>(po.size(), 1));
  const size_t off_cof = take(sizeof(int32_t) * (n_clauses + 1));
  const size_t off_lit = take(sizeof(int32_t) * std::max<size_t>(lits.size(), 1));
  const size_t off_cst = take(sizeof(float) * std::max(n_vslots, 1));
  auto* blob = new std::vector<uint8_t>(o, 0);
  auto put = [&](size_t at, const void* src, size_t bytes) {
    if (bytes) std::memcpy(blob->data() + at, src, bytes);
  };
  put(off_gate, gates.data(), sizeof(tt::GdGate) * gates.size());
  put(off_iv, iv.rng.data(), sizeof(int32_t) * iv.rng.size());
  put(off_aux, aux.rng.data(), sizeof(int32_t) * aux.rng.size());
  put(off_po, po.data(), sizeof(int32_t) * po.size());
  put(off_cof, coff.data(), sizeof(int32_t) * (n_clauses + 1));
  put(off_lit, lits.data(), sizeof(int32_t) * lits.size());
  put(off_cst, cst.data(), sizeof(float) * n_vslots);
  tt_gd* h = new (std::nothrow) tt_gd();
  if (!h) {
    delete blob;
    return TT_ENOMEM;
  }
  hipError_t e = hipMalloc((void**)&h->ws, o);
  if (e != hipSuccess) {
    delete blob;
    delete h;
    g_last_hip = (int)e;
    return TT_ENOMEM;
  }
  const int st = upload_async(h->ws, blob, (hipStream_t)stream);
  if (st != TT_OK) {
    (void)hipStreamSynchronize((hipStream_t)stream);
    (void)hipFree(h->ws);
    delete h;
    return st;
  }
  h->pi_vars = std::move(pi_vars);
  tt::GdArgs& a = h->args;
  a.gate = reinterpret_cast<const tt::GdGate*>(h->ws + off_gate);
  a.iv_rng = reinterpret_cast<const int32_t*>(h->ws + off_iv);
  a.aux_rng = reinterpret_cast<const int32_t*>(h->ws + off_aux);
  a.po = reinterpret_cast<const int32_t*>(h->ws + off_po);
  a.clause_off = reinterpret_cast<const int32_t*>(h->ws + off_cof);
  a.lits = reinterpret_cast<const int32_t*>(h->ws + off_lit);
  a.slot_const = reinterpret_cast<const float*>(h->ws + off_cst);
  a.n_iv = (int32_t)iv.rng.size() - 1;
  a.n_aux = (int32_t)aux.rng.size() - 1;
  a.n_po = (int32_t)po.size() / 2;
  a.n_clauses = n_clauses;
  a.n_pi = n_pi;
  a.n_vslots = n_vslots;
  a.n_slots = n_slots;
  a.words = (n_pi + 63) / 64;
  // the circuit compiled into a kernel of its own (the interpreter serves
  // circuits that are too large or that the run-time compiler rejects)
  {
    tt::GdProgram prog;
    prog.gate = std::move(gates);
    prog.iv_rng = iv.rng;
    prog.aux_rng = aux.rng;
    prog.po = po;
    prog.coff = coff;
    prog.lits = lits;
    prog.cst = cst;
    prog.n_pi = n_pi;
    prog.n_vslots = n_vslots;
    prog.words = a.words;
    if (tt::gd_compile(prog, &h->mod, &h->fn) == 0) h->kernel = TT_GD_COMPILED;
  }
  *out = h;
  return TT_OK;
}

int tt_gd_inputs(const tt_gd* gd, int* n_pi) {
  if (!gd || !n_pi) return TT_EINVAL;
  *n_pi = gd->args.n_pi;
  return TT_OK;
}

int tt_gd_input_vars(const tt_gd* gd, int32_t* h_vars) {
  if (!gd || (!h_vars && !gd->pi_vars.empty())) return TT_EINVAL;
  if (!gd->pi_vars.empty()) std::memcpy(h_vars, gd->pi_vars.data(), sizeof(int32_t) * gd->pi_vars.size());
  return TT_OK;
}

namespace {

// The interpreter on logits updated in place (d_V: initial logits in,
// final logits out).
int gd_run_interpreted(const tt_gd* gd, float* d_V, int batch, float lr, int iters, uint8_t* d_valid,
                       uint64_t* d_solution, hipStream_t s) {
  tt::GdArgs a = gd->args;
  a.V = d_V;
  a.batch = batch;
  a.iters = iters;
  a.lr = lr;
  a.valid = d_valid;
  a.sol = d_solution;
  const bool global_state = (size_t)(2 * a.n_slots) * 64 * sizeof(float) > tt::kGdLdsLimit;
  if (!global_state) {
    TT_HIP(tt::launch_gd_sample(a, s));
    return TT_OK;
  }
  // more slots than a wave's LDS holds: the variables' state goes to a
  // stream-ordered workspace, one column per sample (the temporaries stay
  // in LDS)
  const size_t padded = ((size_t)batch + 63) / 64 * 64;  // one block of rows of 64 per wave
  const size_t nt = (size_t)(a.n_slots - a.n_vslots);
  a.temps_lds = 2 * nt * 64 * sizeof(float) <= tt::kGdTempLdsLimit ? 1 : 0;
  const size_t rows = 2 * (size_t)a.n_vslots + a.n_pi + (a.temps_lds ? 0 : 2 * nt);
  hipError_t e = hipMallocAsync((void**)&a.state, sizeof(float) * rows * padded, s);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    return TT_ENOMEM;
  }
  int st = TT_OK;
  e = tt::launch_gd_sample(a, s);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    st = TT_EHIP;
  }
  e = hipFreeAsync(a.state, s);
  if (st == TT_OK && e != hipSuccess) {
    g_last_hip = (int)e;
    st = TT_EHIP;
  }
  return st;
}

}  // namespace

int tt_gd_run_from(const tt_gd* gd, const float* d_V0, float* d_V, int batch, float lr, int iters, uint8_t* d_valid,
                   uint64_t* d_solution, void* stream) {
  if (!gd || batch < 0 || iters < 0) return TT_EINVAL;
  if (batch == 0) return TT_OK;
  if ((gd->args.n_pi > 0 && !d_V0) || !d_valid || (gd->args.words > 0 && !d_solution)) return TT_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (gd->kernel == TT_GD_COMPILED) {
    // the logits live in registers: read from d_V0, written to d_V if given
    TT_HIP(tt::launch_gd_compiled(gd->fn, d_V0, d_V, batch, lr, iters, d_valid, d_solution, nullptr, 0u, nullptr, 0u,
                                  s));
    return TT_OK;
  }
  // the interpreter updates the logits in place: in d_V (a copy of d_V0
  // first unless they are the same), or in a stream-ordered copy when the
  // final logits are not wanted
  const size_t bytes = sizeof(float) * (size_t)batch * (size_t)gd->args.n_pi;
  float* V = d_V;
  if (!V && bytes) {
    const hipError_t e = hipMallocAsync((void**)&V, bytes, s);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      return TT_ENOMEM;
    }
  }
  int st = TT_OK;
  if (bytes && V != d_V0) {
    const hipError_t e = hipMemcpyAsync(V, d_V0, bytes, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      st = TT_EHIP;
    }
  }
  if (st == TT_OK) st = gd_run_interpreted(gd, V, batch, lr, iters, d_valid, d_solution, s);
  if (V && V != d_V) {
    const hipError_t e = hipFreeAsync(V, s);
    if (st == TT_OK && e != hipSuccess) {
      g_last_hip = (int)e;
      st = TT_EHIP;
    }
  }
  return st;
}

int tt_gd_run(const tt_gd* gd, float* d_V, int batch, float lr, int iters, uint8_t* d_valid, uint64_t* d_solution,
              void* stream) {
  return tt_gd_run_from(gd, d_V, d_V, batch, lr, iters, d_valid, d_solution, stream);
}

int tt_gd_unique(const tt_gd* gd, const uint8_t* d_valid, const uint64_t* d_solution, int batch, uint8_t* d_first,
                 uint32_t* d_count, void* stream) {
  if (!gd || batch < 0) return TT_EINVAL;
  if (batch == 0) return TT_OK;
  if (!d_valid || !d_first || !d_count || (gd->args.words > 0 && !d_solution)) return TT_EINVAL;
  if (batch > (1 << 30)) return TT_ERANGE;  // the table's places (a power of two >= 2 batch) fit 32 bits
  uint32_t cap = 1;
  while (cap < 2u * (uint32_t)batch) cap <<= 1;
  const uint32_t pcap = tt::gd_unique_primary_places(batch);
  hipStream_t s = (hipStream_t)stream;
  int32_t* table = nullptr;  // [pcap] places of the first pass, then [cap] open-addressing places
  hipError_t e = hipMallocAsync((void**)&table, sizeof(int32_t) * ((size_t)pcap + cap), s);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    return TT_ENOMEM;
  }
  int st = TT_OK;
  e = tt::launch_gd_unique(d_valid, d_solution, gd->args.words, batch, table, table + pcap, cap, d_first, d_count,
                           s);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    st = TT_EHIP;
  }
  e = hipFreeAsync(table, s);
  if (st == TT_OK && e != hipSuccess) {
    g_last_hip = (int)e;
    st = TT_EHIP;
  }
  return st;
}


int tt_gd_sample_unique(const tt_gd* gd, const float* d_V0, float* d_V, int batch, float lr, int iters,
                        uint8_t* d_valid, uint64_t* d_solution, uint8_t* d_first, uint32_t* d_count, void* stream) {
  if (!gd || batch < 0 || iters < 0) return TT_EINVAL;
  if (batch == 0) return TT_OK;
  if ((gd->args.n_pi > 0 && !d_V0) || !d_valid || !d_first || !d_count || (gd->args.words > 0 && !d_solution))
    return TT_EINVAL;
  if (batch > (1 << 30)) return TT_ERANGE;
  if (gd->kernel != TT_GD_COMPILED) {
    TT_TRY(tt_gd_run_from(gd, d_V0, d_V, batch, lr, iters, d_valid, d_solution, stream));
    return tt_gd_unique(gd, d_valid, d_solution, batch, d_first, d_count, stream);
  }
  // the filter's tables as in tt_gd_unique; the sampler places the valid
  // samples and clears the second table, the filter's last pass follows
  uint32_t cap = 1;
  while (cap < 2u * (uint32_t)batch) cap <<= 1;
  const uint32_t pcap = tt::gd_unique_primary_places(batch);
  hipStream_t s = (hipStream_t)stream;
  int32_t* table = nullptr;
  hipError_t e = hipMallocAsync((void**)&table, sizeof(int32_t) * ((size_t)pcap + cap), s);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    return TT_ENOMEM;
  }
  int st = TT_OK;
  e = tt::launch_gd_compiled(gd->fn, d_V0, d_V, batch, lr, iters, d_valid, d_solution, table, pcap, table + pcap, cap,
                             s);
  if (e == hipSuccess)
    e = tt::launch_gd_unique_placed(d_valid, d_solution, gd->args.words, batch, table, pcap, table + pcap, cap,
                                    d_first, d_count, s);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    st = TT_EHIP;
  }
  e = hipFreeAsync(table, s);
  if (st == TT_OK && e != hipSuccess) {
    g_last_hip = (int)e;
    st = TT_EHIP;
  }
  return st;
}

int tt_gd_kernel(const tt_gd* gd, int* kernel) {
  if (!gd || !kernel) return TT_EINVAL;
  *kernel = gd->kernel;
  return TT_OK;
}

int tt_gd_set_kernel(tt_gd* gd, int kernel) {
  if (!gd || (kernel != TT_GD_INTERPRETED && kernel != TT_GD_COMPILED)) return TT_EINVAL;
  if (kernel == TT_GD_COMPILED && !gd->fn) return TT_ENOTSUP;
  gd->kernel = kernel;
  return TT_OK;
}

int tt_gd_destroy(tt_gd* gd) {
  if (!gd) return TT_OK;
  int st = TT_OK;
  if (gd->ws || gd->mod)
    if (hipDeviceSynchronize() != hipSuccess) st = TT_EHIP;
  if (gd->ws && hipFree(gd->ws) != hipSuccess) st = TT_EHIP;
  if (gd->mod && hipModuleUnload(gd->mod) != hipSuccess) st = TT_EHIP;
  delete gd;
  return st;
}

int tt_pack(const tt_neuron* h_desc, int n, const uint8_t* d_codes, uint64_t total_codes,
            uint64_t* d_tables, uint64_t total_words, void* stream) {
  TT_TRY(validate_all(h_desc, n));
  if (n == 0) return TT_OK;
  if (!d_codes || !d_tables) return TT_EINVAL;
  TT_TRY(validate_ranges(h_desc, n, total_words));
  hipStream_t s = (hipStream_t)stream;
  std::vector<uint64_t> code_off(n);
  std::vector<int32_t> item_neuron, item_h0;
  uint64_t acc = 0;
  for (int i = 0; i < n; ++i) {
    code_off[i] = acc;
    acc += 1ull << (h_desc[i].F * h_desc[i].b);
    const uint64_t W = words_of(h_desc[i].F, h_desc[i].b);
    for (uint64_t h0 = 0; h0 < W; h0 += 64) {
      item_neuron.push_back(i);
      item_h0.push_back((int32_t)h0);
    }
  }
  if (acc > total_codes) return TT_ERANGE;
  TT_TRY(device_info(nullptr));
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t off_desc = take(sizeof(tt_neuron) * n);
  const size_t off_code = take(sizeof(uint64_t) * n);
  const size_t off_in = take(sizeof(int32_t) * item_neuron.size());
  const size_t off_ih = take(sizeof(int32_t) * item_h0.size());
  auto* blob = new std::vector<uint8_t>(o, 0);
  std::memcpy(blob->data() + off_desc, h_desc, sizeof(tt_neuron) * n);
  std::memcpy(blob->data() + off_code, code_off.data(), sizeof(uint64_t) * n);
  std::memcpy(blob->data() + off_in, item_neuron.data(), sizeof(int32_t) * item_neuron.size());
  std::memcpy(blob->data() + off_ih, item_h0.data(), sizeof(int32_t) * item_h0.size());
  uint8_t* ws = nullptr;
  hipError_t e = hipMallocAsync((void**)&ws, o, s);
  if (e != hipSuccess) {
    delete blob;
    g_last_hip = (int)e;
    return TT_ENOMEM;
  }
  int st = upload_async(ws, blob, s);
  if (st == TT_OK) {
    PackArgs pa{};
    pa.desc = reinterpret_cast<const tt_neuron*>(ws + off_desc);
    pa.codes = d_codes;
    pa.code_off = reinterpret_cast<const uint64_t*>(ws + off_code);
    pa.item_neuron = reinterpret_cast<const int32_t*>(ws + off_in);
    pa.item_h0 = reinterpret_cast<const int32_t*>(ws + off_ih);
    pa.n_items = (int)item_neuron.size();
    pa.words_per_item = 64;
    pa.tables = d_tables;
    e = launch_pack(pa, s);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      st = TT_EHIP;
    }
  }
  e = hipFreeAsync(ws, s);
  if (st == TT_OK && e != hipSuccess) {
    g_last_hip = (int)e;
    st = TT_EHIP;
  }
  return st;
}

// ------------------------------------------------------------- autotune
int tt_autotune(const tt_neuron* h_desc, int n, uint64_t* d_tables, uint64_t total_words,
                const char* cache_path, tt_tune* best) {
  if (!best) return TT_EINVAL;
  TT_TRY(validate_all(h_desc, n));
  TT_TRY(validate_ranges(h_desc, n, total_words));
  TT_TRY(device_info(nullptr));
  // Workload signature: neuron count, total rows and a hash of the shapes.
  uint64_t rows = 0, hsh = 1469598103934665603ull;
  for (int i = 0; i < n; ++i) {
    rows += 1ull << (h_desc[i].F * h_desc[i].b);
    const uint64_t v = (uint64_t)h_desc[i].F | ((uint64_t)h_desc[i].b << 8) | ((uint64_t)h_desc[i].o << 16);
    hsh = (hsh ^ v) * 1099511628211ull;
  }
  char key[200];
  // "hist": timed with the fused histogram on, as the plans run it; "src": a
  // signature of the enumeration kernel sources this library was built from
  std::snprintf(key, sizeof(key), "gfx950:hist:src=%016llx:n=%d:rows=%llu:shape=%016llx",
                (unsigned long long)TT_KERNEL_SIG, n, (unsigned long long)rows, (unsigned long long)hsh);
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "r");
    if (f) {
      char line[512];
      bool hit = false;
      while (std::fgets(line, sizeof(line), f)) {
        char k[240];
        tt_tune t{};
        double us = 0;
        if (std::sscanf(line, "%239s %d %d %d %d %d %lf", k, &t.chunk_words, &t.blocks_per_cu, &t.waves,
                        &t.nontemporal, &t.tile_neurons, &us) == 7 &&
            std::strcmp(k, key) == 0 && check_tune(t) == TT_OK) {
          *best = t;
          hit = true;
        }
      }
      std::fclose(f);
      if (hit) return TT_OK;
    }
  }
  if (n == 0) {
    *best = default_tune();
    return TT_OK;
  }
  hipStream_t s = nullptr;
  TT_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  uint32_t* d_hist = nullptr;
  {
    const hipError_t e = hipMalloc((void**)&d_hist, sizeof(uint32_t) * 8 * (size_t)n);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      (void)hipStreamDestroy(s);
      return TT_ENOMEM;
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  {
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      if (e0) (void)hipEventDestroy(e0);
      (void)hipFree(d_hist);
      (void)hipStreamDestroy(s);
      return TT_EHIP;
    }
  }
  const int chunks[] = {32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384, 32768};
  const int bpcs[] = {1, 2, 3, 4, 6, 8};
  const int waves[] = {4, 8};
  const int nts[] = {0, 1};
  const int tms[] = {8, 16, 32};
  double best_us = 1e300;
  tt_tune best_t = default_tune();
  int st = TT_OK;
  for (int tm : tms)
    for (int c : chunks)
      for (int bpc : bpcs)
        for (int wv : waves)
          for (int nt : nts) {
            tt_tune t{c, bpc, wv, nt, tm};
            tt_plan* p = nullptr;
            st = tt_plan_create(h_desc, n, total_words, &t, TT_PLAN_PERSISTENT, &p);
            if (st != TT_OK) goto done;
            double times[3] = {0, 0, 0};
            for (int rep = 0; rep < 4; ++rep) {
              if (hipEventRecord(e0, s) != hipSuccess) {
                st = TT_EHIP;
                break;
              }
              st = tt_plan_launch(p, d_tables, d_hist, s);
              if (st != TT_OK) break;
              if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                st = TT_EHIP;
                break;
              }
              float ms = 0;
              (void)hipEventElapsedTime(&ms, e0, e1);
              if (rep > 0) times[rep - 1] = ms * 1000.0;
            }
            tt_plan_destroy(p);
            if (st != TT_OK) goto done;
            std::sort(times, times + 3);
            if (times[1] < best_us) {
              best_us = times[1];
              best_t = t;
            }
          }
done:
  (void)hipStreamSynchronize(s);
  (void)hipFree(d_hist);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  if (st != TT_OK) return st;
  *best = best_t;
  if (cache_path) {
    FILE* f = std::fopen(cache_path, "a");
    if (f) {
      std::fprintf(f, "%s %d %d %d %d %d %.3f\n", key, best_t.chunk_words, best_t.blocks_per_cu, best_t.waves,
                   best_t.nontemporal, best_t.tile_neurons, best_us);
      std::fclose(f);
    }
  }
  return TT_OK;
}

// ---------------------------------------------------------- learned screen
#define TT_HIPCALL(expr)         \
  do {                           \
    hipError_t e_ = (expr);      \
    if (e_ != hipSuccess) {      \
      g_last_hip = (int)e_;      \
      return TT_EHIP;            \
    }                            \
  } while (0)

int tt_enumerate_device(const tt_neuron* d_desc, int n, const uint8_t* d_active, uint64_t* d_tables,
                        uint64_t total_words, uint32_t* d_status, void* stream) {
  if (n < 0 || (n > 0 && (!d_desc || !d_tables))) return TT_EINVAL;
  TT_HIPCALL(small_enumerate(d_desc, n, d_active, d_tables, total_words, d_status, (hipStream_t)stream));
  return TT_OK;
}

int tt_support_device(const tt_neuron* d_desc, int n, const uint64_t* d_tables, uint64_t total_words,
                      uint8_t* d_support, uint32_t* d_hist, uint32_t* d_status, void* stream) {
  if (n < 0 || (n > 0 && (!d_desc || !d_tables || (!d_support && !d_hist)))) return TT_EINVAL;
  TT_HIPCALL(small_support(d_desc, n, d_tables, total_words, d_support, d_hist, d_status, (hipStream_t)stream));
  return TT_OK;
}

int tt_screen_features(const tt_neuron* d_desc, int n, uint16_t* d_x, void* stream) {
  if (n < 0 || (n > 0 && (!d_desc || !d_x))) return TT_EINVAL;
  TT_HIPCALL(screen_features(d_desc, n, d_x, (hipStream_t)stream));
  return TT_OK;
}

int tt_screen_labels(const tt_neuron* d_desc, int n, const uint8_t* d_support, const uint32_t* d_hist, float* d_y,
                     float* d_m, float* d_h, void* stream) {
  if (n < 0 || (n > 0 && (!d_desc || !d_support || !d_hist || !d_y || !d_m || !d_h))) return TT_EINVAL;
  TT_HIPCALL(screen_labels(d_desc, n, d_support, d_hist, d_y, d_m, d_h, (hipStream_t)stream));
  return TT_OK;
}

int tt_mlp_forward(const uint16_t* d_x, int batch, int in, const uint16_t* d_w, const float* d_bias, int out,
                   int relu, uint16_t* d_y_bf16, float* d_y_f32, void* stream) {
  if (batch < 0 || in < 1 || out < 1 || (batch > 0 && (!d_x || !d_w || (!d_y_bf16 && !d_y_f32)))) return TT_EINVAL;
  TT_HIPCALL(mlp_forward(d_x, batch, in, d_w, d_bias, out, relu, d_y_bf16, d_y_f32, (hipStream_t)stream));
  return TT_OK;
}

int tt_mlp_infer(const uint16_t* d_x, int n, const uint16_t* d_w1, const float* d_b1, const uint16_t* d_w2,
                 const float* d_b2, const uint16_t* d_w3, const float* d_b3, const uint16_t* d_w4, const float* d_b4,
                 float* d_logits, void* stream) {
  if (n < 0) return TT_EINVAL;
  if (n == 0) return TT_OK;
  const uint16_t* w[4] = {d_w1, d_w2, d_w3, d_w4};
  const float* b[4] = {d_b1, d_b2, d_b3, d_b4};
  if (!d_x || !d_logits || (uintptr_t)d_x % 16) return TT_EINVAL;
  for (int l = 0; l < 4; ++l)
    if (!w[l] || (uintptr_t)w[l] % 16 || (uintptr_t)b[l] % 16) return TT_EINVAL;
  TT_HIPCALL(mlp_infer(d_x, n, w, b, d_logits, (hipStream_t)stream));
  return TT_OK;
}

int tt_mlp_backward(const uint16_t* d_dy, int batch, int out, const uint16_t* d_w, int in, const uint16_t* d_x,
                    int relu_mask, uint16_t* d_dx, float* d_dw, float* d_db, float* d_scratch, size_t scratch_floats,
                    void* stream) {
  if (batch < 1 || in < 1 || out < 1 || !d_dy) return TT_EINVAL;
  if ((d_dx && !d_w) || ((d_dw || d_db) && !d_x) || ((d_db || d_dw) && !d_scratch) || (relu_mask && !d_x))
    return TT_EINVAL;
  // a scratch, when given, must have the full size (the input gradient uses it too)
  if (d_scratch && scratch_floats < mlp_backward_scratch_floats(batch, in > out ? in : out)) return TT_ERANGE;
  TT_HIPCALL(mlp_backward(d_dy, batch, out, d_w, in, d_x, relu_mask, d_dx, d_dw, d_db, d_scratch,
                          (hipStream_t)stream));
  return TT_OK;
}

int tt_cast_bf16(const float* d_x, uint16_t* d_y, size_t n, void* stream) {
  if (n > 0 && (!d_x || !d_y)) return TT_EINVAL;
  TT_HIPCALL(cast_bf16(d_x, d_y, n, (hipStream_t)stream));
  return TT_OK;
}

size_t tt_mlp_scratch_floats(int batch, int dim) {
  const size_t c = batch > 0 && dim > 0 ? mlp_backward_scratch_floats(batch, dim) : 0;
  return c > 64 ? c : 64;
}

int tt_mlp_loss(const float* d_z, int batch, const float* d_y, const float* d_m, const float* d_h, uint16_t* d_dz,
                float* d_loss, float* d_scratch, void* stream) {
  if (batch < 1 || !d_z || !d_y || !d_m || !d_h || !d_dz || !d_loss || !d_scratch) return TT_EINVAL;
  TT_HIPCALL(mlp_loss(d_z, batch, d_y, d_m, d_h, d_dz, d_loss, d_scratch, (hipStream_t)stream));
  return TT_OK;
}

int tt_adam_step_multi(int count, float* const* h_d_p, const float* const* h_d_g, float* const* h_d_m,
                       float* const* h_d_v, uint16_t* const* h_d_p_bf16, const size_t* h_n, float lr, float beta1,
                       float beta2, float eps, int step, void* stream) {
  if (count < 0 || count > kAdamMaxTensors || step < 1) return TT_EINVAL;
  if (count == 0) return TT_OK;
  if (!h_d_p || !h_d_g || !h_d_m || !h_d_v || !h_n) return TT_EINVAL;
  for (int t = 0; t < count; ++t)
    if (h_n[t] > 0 && (!h_d_p[t] || !h_d_g[t] || !h_d_m[t] || !h_d_v[t])) return TT_EINVAL;
  const float bc1 = 1.0f - (float)std::pow((double)beta1, (double)step);
  const float bc2 = 1.0f - (float)std::pow((double)beta2, (double)step);
  TT_HIPCALL(adam_step_multi(count, h_d_p, h_d_g, h_d_m, h_d_v, h_d_p_bf16, h_n, lr, beta1, beta2, eps, bc1, bc2,
                             (hipStream_t)stream));
  return TT_OK;
}

int tt_adam_step(float* d_p, const float* d_g, float* d_m, float* d_v, uint16_t* d_p_bf16, size_t n, float lr,
                 float beta1, float beta2, float eps, int step, void* stream) {
  if (step < 1 || (n > 0 && (!d_p || !d_g || !d_m || !d_v))) return TT_EINVAL;
  const float bc1 = 1.0f - (float)std::pow((double)beta1, (double)step);
  const float bc2 = 1.0f - (float)std::pow((double)beta2, (double)step);
  TT_HIPCALL(adam_step(d_p, d_g, d_m, d_v, d_p_bf16, n, lr, beta1, beta2, eps, bc1, bc2, (hipStream_t)stream));
  return TT_OK;
}

namespace {
struct ScreenWork {
  size_t res, mask, mode, accept, list, count, total;
};
ScreenWork screen_work_layout(int n) {
  ScreenWork w{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  w.res = take(sizeof(tt_neuron) * (size_t)n);
  w.mask = take((size_t)n);
  w.mode = take((size_t)n);
  w.accept = take((size_t)n);
  w.list = take(sizeof(int32_t) * (size_t)n);
  w.count = take(sizeof(uint32_t) * 4);
  w.total = o;
  return w;
}
}  // namespace

size_t tt_screen_work_bytes(int n) { return n > 0 ? screen_work_layout(n).total : 0; }

int tt_screen_run(const tt_neuron* d_desc, int n, const float* d_logits, float tau, const uint8_t* d_force_mask,
                  uint64_t* d_tables, uint64_t total_words, uint8_t* d_support, uint32_t* d_hist, uint8_t* d_mask,
                  uint8_t* d_accept, void* d_work, uint32_t* d_status, void* stream) {
  if (n < 0) return TT_EINVAL;
  if (n == 0) return TT_OK;
  if (!d_desc || !d_tables || !d_support || !d_hist || !d_work) return TT_EINVAL;
  const bool plain = !d_logits && !d_force_mask;
  if (d_logits && !d_force_mask && !(tau > 0.f && tau < 1.f)) return TT_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const ScreenWork w = screen_work_layout(n);
  uint8_t* ws = static_cast<uint8_t*>(d_work);
  FusedArgs fa{};
  fa.desc = d_desc;
  fa.n = n;
  fa.plain = plain ? 1 : 0;
  fa.logits = d_logits;
  fa.tau_logit = (plain || d_force_mask) ? 0.f : (float)std::log((double)tau / (1.0 - (double)tau));
  fa.force_mask = d_force_mask;
  fa.tables = d_tables;
  fa.total_words = total_words;
  fa.support = d_support;
  fa.hist = d_hist;
  fa.res = reinterpret_cast<tt_neuron*>(ws + w.res);
  fa.mask = ws + w.mask;
  fa.mode = ws + w.mode;
  fa.accept = ws + w.accept;
  fa.status = d_status;
  fa.mask_out = d_mask;
  fa.accept_out = d_accept;
  fa.list = reinterpret_cast<int32_t*>(ws + w.list);
  fa.list_count = reinterpret_cast<uint32_t*>(ws + w.count);
  TT_HIPCALL(screen_fused(fa, s));
  return TT_OK;
}

size_t tt_screen_infer_work_bytes(int n) {
  if (n <= 0 || (n + tt::kGateSpan - 1) / tt::kGateSpan > tt::kGateMaxSpans) return 0;
  return sizeof(int32_t) * tt::gate_work_ints(n);
}

int tt_screen_infer(const tt_neuron* d_desc, int n, int gated, const uint16_t* d_w1, const float* d_b1,
                    const uint16_t* d_w2, const float* d_b2, const uint16_t* d_w3, const float* d_b3,
                    const uint16_t* d_w4, const float* d_b4, float* d_logits, void* d_work, void* stream) {
  if (n < 0 || (gated != 0 && gated != 1)) return TT_EINVAL;
  if (n == 0) return TT_OK;
  if (!d_desc || !d_logits || (uintptr_t)d_desc % 16) return TT_EINVAL;
  const uint16_t* w[4] = {d_w1, d_w2, d_w3, d_w4};
  const float* b[4] = {d_b1, d_b2, d_b3, d_b4};
  for (int l = 0; l < 4; ++l)
    if (!w[l] || (uintptr_t)w[l] % 16 || (uintptr_t)b[l] % 16) return TT_EINVAL;
  if (d_work && (uintptr_t)d_work % 4) return TT_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (!gated || (n + tt::kGateSpan - 1) / tt::kGateSpan > tt::kGateMaxSpans) {
    TT_HIPCALL(mlp_infer(nullptr, n, w, b, d_logits, s, d_desc, gated));
    return TT_OK;
  }
  // gated: the candidates compacted first (stream-ordered list), then one
  // block per CU over it, so the gated rows are spread evenly
  int cus = 0;
  TT_TRY(device_info(&cus));
  int32_t* work = static_cast<int32_t*>(d_work);
  hipError_t e = hipSuccess;
  if (!work) {
    e = hipMallocAsync((void**)&work, tt_screen_infer_work_bytes(n), s);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      return TT_ENOMEM;
    }
  }
  int st = TT_OK;
  e = tt::mlp_infer_gated_list(d_desc, n, w, b, d_logits, work, cus, s);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    st = TT_EHIP;
  }
  if (!d_work) {
    e = hipFreeAsync(work, s);
    if (st == TT_OK && e != hipSuccess) {
      g_last_hip = (int)e;
      st = TT_EHIP;
    }
  }
  return st;
}

int tt_screen_expand(const tt_neuron* d_desc, int n, const void* d_work, const uint64_t* d_screened,
                     uint64_t* d_full, void* stream) {
  if (n < 0) return TT_EINVAL;
  if (n == 0) return TT_OK;
  if (!d_desc || !d_work || !d_screened || !d_full) return TT_EINVAL;
  const ScreenWork w = screen_work_layout(n);
  const uint8_t* ws = static_cast<const uint8_t*>(d_work);
  TT_HIPCALL(screen_expand(d_desc, n, ws + w.mask, ws + w.mode, ws + w.accept,
                           reinterpret_cast<const tt_neuron*>(ws + w.res), d_screened, d_full,
                           (hipStream_t)stream));
  return TT_OK;
}

}  // extern "C"
