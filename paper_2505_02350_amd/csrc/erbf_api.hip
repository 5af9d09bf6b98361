// C ABI layer: context, workspace layout, argument checks and call sequencing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "erbf.h"
#include "erbf_internal.h"
#include "erbf_launch.h"

using namespace erbf;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(ERBF_ERR_HIP, std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}

#define HIP_TRY(expr, where)                   \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  int n_levels_total = 0;
  int cap_total = 0;
  int tiles_total = 0;
  int max_level_tiles = 0;
  int64_t pts_total = 0;
  int64_t cand_cap = 0;
  int64_t init_words = 0;   // candidate mask words of the inscribed-sphere initialisation
  int64_t init_cand = 0;    // its candidate list capacity: points of the largest shape
  int scan_blocks = 0;
  int radix_nb = 0;
  int hit_cap = 0;   // tile slots kept per kernel by the count pass (0: the emit pass walks)
  size_t off_levels, off_shapes, off_kshape, off_slot_tile, off_tile_map, off_tile_start, off_tile_cnt,
      off_tile_start64, off_kslot, off_sort_keys[2],
      off_sort_vals[2], off_kj, off_rhist, off_rhist_ex, off_tile_keys, off_tile_e, off_items, off_kcnt, off_hits, off_tile_order, off_order_hist, off_kstart, off_kblock, off_kblock_ex, off_sort_j[2],
      off_partials,
      off_scan, off_rflags, off_rexcl, off_rec, off_G, off_tstat, off_tile_pbwd,
      off_counters, off_tickets, off_stat_part, off_stat_ab, off_prune_flag, off_sched_held, off_b_l2, off_b_abs, off_b_id, off_b_pf,
      off_b_shape, off_hist, off_cand, off_keep, off_misc, off_init, off_samp_pos, off_samp_start, off_samp_slot,
      off_samp_slots, off_samp_f, off_samp_c, off_samp_pb, off_sel;
  int64_t samp_total = 0, samp_start_total = 0, samp_tiles = 0;
  size_t bytes = 0;
};

int validate_config(const erbf_config* cfg) {
  if (!cfg) return fail(ERBF_ERR_INVALID_ARG, "config is NULL");
  if (cfg->n_shapes < 1 || cfg->n_shapes > ERBF_MAX_SHAPES)
    return fail(ERBF_ERR_INVALID_ARG, "n_shapes out of range");
  if (!cfg->shapes) return fail(ERBF_ERR_INVALID_ARG, "shapes is NULL");
  if (!(cfg->cull_k > 0.f) || !std::isfinite(cfg->cull_k)) return fail(ERBF_ERR_INVALID_ARG, "cull_k must be > 0");
  if (cfg->weight_map != ERBF_WEIGHT_SIGNED_SQUARE && cfg->weight_map != ERBF_WEIGHT_LINEAR)
    return fail(ERBF_ERR_INVALID_ARG, "unknown weight_map");
  if (cfg->orientation != ERBF_ORIENT_QUATERNION && cfg->orientation != ERBF_ORIENT_EULER)
    return fail(ERBF_ERR_INVALID_ARG, "unknown orientation");
  if (cfg->batch_cap < 0 || cfg->batch_cap > (1 << 28)) return fail(ERBF_ERR_INVALID_ARG, "batch_cap out of range");
  if (cfg->pair_cap < 1 || cfg->pair_cap > (int64_t)INT32_MAX)
    return fail(ERBF_ERR_INVALID_ARG, "pair_cap must be in [1, 2^31)");
  int64_t cap = 0, tiles = 0;
  for (int b = 0; b < cfg->n_shapes; ++b) {
    const erbf_shape_desc& s = cfg->shapes[b];
    if (s.n_levels < 1 || s.n_levels > ERBF_MAX_LEVELS) return fail(ERBF_ERR_INVALID_ARG, "n_levels out of range");
    if (s.m_cap < 1) return fail(ERBF_ERR_INVALID_ARG, "m_cap must be >= 1");
    cap += s.m_cap;
    for (int l = 0; l < s.n_levels; ++l) {
      const int n = s.level_n[l];
      if (n < 1 || n > 2048) return fail(ERBF_ERR_INVALID_ARG, "level_n out of range");
      if (s.level_samples[l] < 0 || s.level_samples[l] > (1 << 26))
        return fail(ERBF_ERR_INVALID_ARG, "level_samples out of range");
      const int64_t nt = (n + kTile - 1) / kTile;
      tiles += nt * nt * nt;
    }
  }
  if (cap > (int64_t)INT32_MAX / 16) return fail(ERBF_ERR_INVALID_ARG, "total kernel capacity too large");
  if (tiles > (int64_t)INT32_MAX / 4) return fail(ERBF_ERR_INVALID_ARG, "too many tiles");
  return ERBF_OK;
}

Layout make_layout(const erbf_config* cfg) {
  Layout L;
  for (int b = 0; b < cfg->n_shapes; ++b) {
    const erbf_shape_desc& s = cfg->shapes[b];
    L.cap_total += s.m_cap;
    L.n_levels_total += s.n_levels;
    for (int l = 0; l < s.n_levels; ++l) {
      const int n = s.level_n[l];
      const int nt = (n + kTile - 1) / kTile;
      L.tiles_total += nt * nt * nt;
      L.max_level_tiles = std::max(L.max_level_tiles, nt * nt * nt);
      if (s.level_samples[l] > 0) {
        L.pts_total += s.level_samples[l];
        L.samp_total += s.level_samples[l];
        L.samp_start_total += (int64_t)nt * nt * nt + 1;
        L.samp_tiles += (int64_t)nt * nt * nt;
      } else {
        L.pts_total += (int64_t)n * n * n;
      }
    }
  }
  L.cand_cap = L.pts_total / 20 + 1024;
  // radix-sort blocks: about 4096 bucket entries each at full capacity
  L.radix_nb = (int)std::min<int64_t>(1024, std::max<int64_t>(32, (cfg->pair_cap + 4095) / 4096));
  L.scan_blocks = (std::max(std::max(L.tiles_total, L.cap_total), 256 * L.radix_nb) + 1) / 1024 + 2;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  L.off_levels = take(sizeof(LevelDev) * L.n_levels_total);
  L.off_shapes = take(sizeof(ShapeDev) * cfg->n_shapes);
  L.off_kshape = take(sizeof(int32_t) * L.cap_total);
  L.off_slot_tile = take(sizeof(int2) * L.tiles_total);
  L.off_tile_map = take(sizeof(int32_t) * L.tiles_total);
  L.off_tile_start = take(sizeof(int32_t) * (L.tiles_total + 1));
  L.off_tile_cnt = take(sizeof(int32_t) * (L.tiles_total + 1));
  L.off_tile_start64 = take(sizeof(int64_t) * (L.tiles_total + 1));
  for (int k = 0; k < 2; ++k) {
    L.off_sort_keys[k] = take(sizeof(int32_t) * cfg->pair_cap);
    L.off_sort_vals[k] = take(sizeof(int32_t) * cfg->pair_cap);
    L.off_sort_j[k] = take(sizeof(int32_t) * cfg->pair_cap);
  }
  L.off_kj = take(sizeof(int32_t) * cfg->pair_cap);
  L.off_kslot = take(sizeof(int32_t) * cfg->pair_cap);
  L.off_tile_keys = take(sizeof(int32_t) * cfg->pair_cap);
  L.off_tile_e = take(sizeof(int32_t) * cfg->pair_cap);
  L.off_rhist = take(sizeof(int32_t) * (256 * (size_t)L.radix_nb + 1));
  L.off_rhist_ex = take(sizeof(int32_t) * (256 * (size_t)L.radix_nb + 256));
  L.off_items = take(sizeof(int32_t) * cfg->pair_cap);
  L.off_kcnt = take(sizeof(int32_t) * (L.cap_total + 1));
  L.off_tile_order = take(sizeof(int32_t) * ((size_t)L.tiles_total + 1));
  L.off_order_hist = take(sizeof(int32_t) * kOrderClasses * ((size_t)L.tiles_total / 256 + 2));
  // the count pass keeps each kernel's first hit_cap tile slots, so the emit
  // pass copies them instead of walking the box again; sized to at most
  // twice the list capacity
  L.hit_cap = (int)std::min<int64_t>(kHitCapMax, 2 * cfg->pair_cap / std::max(L.cap_total, 1));
  if (L.hit_cap < 16) L.hit_cap = 0;
  L.off_hits = take(sizeof(int32_t) * (size_t)L.cap_total * (size_t)L.hit_cap + 4);
  L.off_kstart = take(sizeof(int64_t) * (L.cap_total + 1));
  L.off_kblock = take(sizeof(int32_t) * (L.cap_total / 4 + 1));
  L.off_kblock_ex = take(sizeof(int64_t) * (L.cap_total / 4 + 2));
  L.off_partials = take(sizeof(float2) * 5 * cfg->pair_cap);
  L.off_scan = take(sizeof(int64_t) * L.scan_blocks);
  L.off_rflags = take(sizeof(int32_t) * (L.max_level_tiles + 1));
  L.off_rexcl = take(sizeof(int32_t) * (L.max_level_tiles + 1));
  L.off_rec = take(sizeof(float4) * 3 * L.cap_total);
  L.off_G = take(sizeof(float) * L.pts_total);
  L.off_tstat = take(sizeof(TileStat) * L.tiles_total);
  L.off_tile_pbwd = take(sizeof(int64_t) * L.tiles_total);
  L.off_counters = take(sizeof(int64_t) * 8);
  L.off_tickets = take(sizeof(uint32_t) * (cfg->n_shapes + 1));
  L.off_stat_part = take(sizeof(StatPart) * kStatParts * cfg->n_shapes);
  L.off_stat_ab = take(sizeof(double2) * cfg->n_shapes);
  L.off_prune_flag = take(sizeof(int32_t) * cfg->n_shapes);
  L.off_sched_held = take(sizeof(int32_t) * cfg->n_shapes);
  const size_t bc = (size_t)std::max(cfg->batch_cap, 1);
  L.off_b_l2 = take(sizeof(double) * bc);
  L.off_b_abs = take(sizeof(float) * bc);
  L.off_b_id = take(sizeof(int32_t) * bc);
  L.off_b_pf = take(sizeof(int32_t) * bc);
  L.off_b_shape = take(sizeof(int32_t) * bc);
  L.off_hist = take(sizeof(uint32_t) * 65536);
  L.off_cand = take(sizeof(int64_t) * L.cand_cap);
  L.off_keep = take(sizeof(int64_t) * L.cand_cap);
  L.off_misc = take(sizeof(int32_t) * 64);
  L.init_words = L.pts_total / 32 + 1;
  for (int b = 0; b < cfg->n_shapes; ++b) {
    int64_t np = 0;
    for (int l = 0; l < cfg->shapes[b].n_levels; ++l) {
      const int64_t n = cfg->shapes[b].level_n[l];
      np += cfg->shapes[b].level_samples[l] > 0 ? cfg->shapes[b].level_samples[l] : n * n * n;
    }
    L.init_cand = std::max(L.init_cand, np + 1);
  }
  L.off_init = take(sizeof(uint32_t) * ((size_t)L.init_words + 4 * (size_t)L.init_cand + 8));
  L.off_samp_pos = take(sizeof(float4) * (size_t)std::max<int64_t>(L.samp_total, 1));
  L.off_samp_start = take(sizeof(int32_t) * (size_t)std::max<int64_t>(L.samp_start_total, 1));
  L.off_samp_slot = take(sizeof(int32_t) * (size_t)std::max<int64_t>(L.samp_total, 1));
  L.off_samp_slots = take(sizeof(int32_t) * (size_t)std::max<int64_t>(L.samp_tiles, 1));
  L.off_sel = take(sizeof(int32_t) * (size_t)std::max(L.tiles_total, 1));
  L.off_samp_f = take(sizeof(float) * kSampSplitMax * (size_t)std::max<int64_t>(L.samp_total, 1));
  L.off_samp_c = take(sizeof(int32_t) * kSampSplitMax * (size_t)std::max<int64_t>(L.samp_total, 1));
  L.off_samp_pb = take(sizeof(int64_t) * kSampSplitMax * (size_t)std::max<int64_t>(L.samp_tiles, 1));
  L.bytes = o;
  return L;
}

}  // namespace

struct erbf_ctx {
  int device = 0;
  erbf_config cfg{};
  std::vector<erbf_shape_desc> shape_desc;
  Layout lay;
  Dev D{};
  std::vector<LevelDev> lv;
  std::vector<ShapeDev> sh;
  int slots_used = 0;
  int64_t samp_used = 0, samp_start_used = 0;   // sample arrays handed to registered levels
  int32_t* rflags = nullptr;
  int32_t* rexcl = nullptr;
  // optional kernel timing: six events per recorded call (start/stop of the
  // forward, backward-tiles and backward-reduce kernels)
  std::vector<hipEvent_t> tev;
  std::vector<uint8_t> tshared;   // per call: which intervals start at the previous kernel's stop event
  int t_max = 0, t_used = 0;
  ~erbf_ctx() {
    for (hipEvent_t e : tev) (void)hipEventDestroy(e);
  }
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

constexpr int kEvPerCall = 6;

// events of the current timed call (nullptr when not timing)
const hipEvent_t* tev_call(erbf_ctx* c) {
  if (c->t_used >= c->t_max) return nullptr;
  return &c->tev[kEvPerCall * c->t_used];
}

int check_params(const erbf_ctx* ctx, const erbf_params* p) {
  if (!ctx) return fail(ERBF_ERR_INVALID_ARG, "ctx is NULL");
  if (!p || !p->p || !p->m_dev) return fail(ERBF_ERR_INVALID_ARG, "params (p, m_dev) must be non-NULL");
  if (ctx->slots_used <= 0) return fail(ERBF_ERR_STATE, "no grid level registered (call erbf_refine_level)");
  return ERBF_OK;
}

}  // namespace

extern "C" {

int32_t erbf_abi_version(void) { return ERBF_ABI_VERSION; }

const char* erbf_last_error(void) { return g_last_error.c_str(); }

int erbf_workspace_size(const erbf_config* cfg, size_t* bytes) {
  int rc = validate_config(cfg);
  if (rc) return rc;
  if (!bytes) return fail(ERBF_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = make_layout(cfg).bytes;
  return ERBF_OK;
}

int erbf_ctx_create(int device, const erbf_config* cfg, void* workspace, size_t bytes, erbf_ctx** out) {
  int rc = validate_config(cfg);
  if (rc) return rc;
  if (!out) return fail(ERBF_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!workspace) return fail(ERBF_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(ERBF_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  Layout lay = make_layout(cfg);
  if (bytes < lay.bytes)
    return fail(ERBF_ERR_WORKSPACE, "workspace too small: need " + std::to_string(lay.bytes) + " bytes");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(ERBF_ERR_INVALID_ARG, "bad device index");
  DeviceGuard guard(device);

  erbf_ctx* c = new (std::nothrow) erbf_ctx();
  if (!c) return fail(ERBF_ERR_INVALID_ARG, "out of host memory");
  c->device = device;
  c->cfg = *cfg;
  c->shape_desc.assign(cfg->shapes, cfg->shapes + cfg->n_shapes);
  c->cfg.shapes = c->shape_desc.data();
  c->lay = lay;
  char* w = static_cast<char*>(workspace);
  Dev& D = c->D;
  D.levels = reinterpret_cast<LevelDev*>(w + lay.off_levels);
  D.shapes = reinterpret_cast<ShapeDev*>(w + lay.off_shapes);
  D.kshape = reinterpret_cast<int32_t*>(w + lay.off_kshape);
  D.slot_tile = reinterpret_cast<int2*>(w + lay.off_slot_tile);
  D.tile_map = reinterpret_cast<int32_t*>(w + lay.off_tile_map);
  D.tile_start = reinterpret_cast<int32_t*>(w + lay.off_tile_start);
  D.tile_cnt = reinterpret_cast<int32_t*>(w + lay.off_tile_cnt);
  D.tile_start64 = reinterpret_cast<int64_t*>(w + lay.off_tile_start64);
  for (int k = 0; k < 2; ++k) {
    D.sort_keys[k] = reinterpret_cast<int32_t*>(w + lay.off_sort_keys[k]);
    D.sort_vals[k] = reinterpret_cast<int32_t*>(w + lay.off_sort_vals[k]);
    D.sort_j[k] = reinterpret_cast<int32_t*>(w + lay.off_sort_j[k]);
  }
  D.kj = reinterpret_cast<int32_t*>(w + lay.off_kj);
  D.kslot = reinterpret_cast<int32_t*>(w + lay.off_kslot);
  D.tile_keys = reinterpret_cast<int32_t*>(w + lay.off_tile_keys);
  D.tile_e = reinterpret_cast<int32_t*>(w + lay.off_tile_e);
  D.rhist = reinterpret_cast<int32_t*>(w + lay.off_rhist);
  D.rhist_ex = reinterpret_cast<int32_t*>(w + lay.off_rhist_ex);
  D.items = reinterpret_cast<int32_t*>(w + lay.off_items);
  D.kcnt = reinterpret_cast<int32_t*>(w + lay.off_kcnt);
  D.tile_order = reinterpret_cast<int32_t*>(w + lay.off_tile_order);
  D.order_hist = reinterpret_cast<int32_t*>(w + lay.off_order_hist);
  D.hits = reinterpret_cast<int32_t*>(w + lay.off_hits);
  D.hit_cap = lay.hit_cap;
  D.kstart = reinterpret_cast<int64_t*>(w + lay.off_kstart);
  D.kblock = reinterpret_cast<int32_t*>(w + lay.off_kblock);
  D.kblock_ex = reinterpret_cast<int64_t*>(w + lay.off_kblock_ex);
  D.partials = reinterpret_cast<float2*>(w + lay.off_partials);
  D.scan_blocks = reinterpret_cast<int32_t*>(w + lay.off_scan);
  c->rflags = reinterpret_cast<int32_t*>(w + lay.off_rflags);
  c->rexcl = reinterpret_cast<int32_t*>(w + lay.off_rexcl);
  D.rec = reinterpret_cast<float4*>(w + lay.off_rec);
  D.G = reinterpret_cast<float*>(w + lay.off_G);
  D.tstat = reinterpret_cast<TileStat*>(w + lay.off_tstat);
  D.tile_pbwd = reinterpret_cast<int64_t*>(w + lay.off_tile_pbwd);
  D.counters = reinterpret_cast<int64_t*>(w + lay.off_counters);
  D.tickets = reinterpret_cast<uint32_t*>(w + lay.off_tickets);
  D.stat_part = reinterpret_cast<StatPart*>(w + lay.off_stat_part);
  D.stat_ab = reinterpret_cast<double2*>(w + lay.off_stat_ab);
  D.prune_flag = reinterpret_cast<int32_t*>(w + lay.off_prune_flag);
  D.sched_held = reinterpret_cast<int32_t*>(w + lay.off_sched_held);
  D.b_l2 = reinterpret_cast<double*>(w + lay.off_b_l2);
  D.b_abs = reinterpret_cast<float*>(w + lay.off_b_abs);
  D.b_id = reinterpret_cast<int32_t*>(w + lay.off_b_id);
  D.b_pf = reinterpret_cast<int32_t*>(w + lay.off_b_pf);
  D.b_shape = reinterpret_cast<int32_t*>(w + lay.off_b_shape);
  D.batch_cap = cfg->batch_cap;
  D.n_levels_total = lay.n_levels_total;
  D.seed_hist = reinterpret_cast<uint32_t*>(w + lay.off_hist);
  D.seed_cand = reinterpret_cast<int64_t*>(w + lay.off_cand);
  D.seed_keep = reinterpret_cast<int64_t*>(w + lay.off_keep);
  D.seed_misc = reinterpret_cast<int32_t*>(w + lay.off_misc);
  D.init_scratch = reinterpret_cast<uint32_t*>(w + lay.off_init);
  D.samp_pos = reinterpret_cast<float4*>(w + lay.off_samp_pos);
  D.samp_start = reinterpret_cast<int32_t*>(w + lay.off_samp_start);
  D.samp_slot = reinterpret_cast<int32_t*>(w + lay.off_samp_slot);
  D.samp_slots = reinterpret_cast<int32_t*>(w + lay.off_samp_slots);
  D.n_samp_slots = 0;
  D.samp_f = reinterpret_cast<float*>(w + lay.off_samp_f);
  D.sel_buf = reinterpret_cast<int32_t*>(w + lay.off_sel);
  D.tile_sel = nullptr;
  D.samp_c = reinterpret_cast<int32_t*>(w + lay.off_samp_c);
  D.samp_pb = reinterpret_cast<int64_t*>(w + lay.off_samp_pb);
  D.init_words = lay.init_words;
  D.init_cand_cap = lay.init_cand;
  D.cand_cap = lay.cand_cap;
  D.pair_cap = cfg->pair_cap;
  D.radix_nb = lay.radix_nb;
  D.cap_total = lay.cap_total;
  D.tiles_total = lay.tiles_total;
  // slots (the filler slot tiles_total included) and kernel ids both fit in
  // 16 bits: one 32-bit key per entry carries both through the sort
  D.packed_keys = lay.cap_total <= 65536 && lay.tiles_total <= 65535;
  D.n_shapes = cfg->n_shapes;
  D.cull_k = cfg->cull_k;
  D.weight_map = cfg->weight_map;
  D.orientation = cfg->orientation;
  D.variant = 0;
  D.slot_chunk = 8;
  D.samp_split = 16;
  D.fwd_chunk = 256;
  D.bwd_waves = 4;
  D.tile_order_on = 1;
  {
    int max_cap = 1;
    for (int b = 0; b < cfg->n_shapes; ++b) max_cap = std::max(max_cap, cfg->shapes[b].m_cap);
    D.rank_words = (max_cap + 31) / 32;
    D.bucket_rank = 0;   // the radix sort: the ranked lists' placement atomics contend across XCDs
  }
  {
    hipDeviceProp_t prop;
    const hipError_t pe = hipGetDeviceProperties(&prop, device);
    D.persistent_wgs = (pe == hipSuccess && prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256) * 8;
  }

  // host mirrors of the level and shape tables
  std::vector<int32_t> kshape(lay.cap_total);
  int kbase = 0, tmap = 0, li = 0;
  int64_t pbase = 0;
  for (int b = 0; b < cfg->n_shapes; ++b) {
    const erbf_shape_desc& s = cfg->shapes[b];
    ShapeDev sd{};
    sd.kbase = kbase;
    sd.cap = s.m_cap;
    sd.lvl0 = li;
    sd.n_active = 0;
    sd.slot0 = 0;
    sd.n_slots = 0;
    sd.pt_base = pbase;
    for (int l = 0; l < s.n_levels; ++l, ++li) {
      LevelDev L{};
      L.n = s.level_n[l];
      L.nt = (L.n + kTile - 1) / kTile;
      L.shape = b;
      L.slot0 = 0;
      L.n_slots = 0;
      L.tmap0 = tmap;
      L.pt_base = pbase;
      L.h = 2.0f / (float)L.n;
      L.lo = -1.0f + 1.0f / (float)L.n;
      L.kind = s.level_samples[l] > 0 ? kLevelSamples : kLevelGrid;
      L.npts = L.kind == kLevelSamples ? (int64_t)s.level_samples[l] : (int64_t)L.n * L.n * L.n;
      // grid tiles: their points' box (plus rounding); sample tiles: their cells
      L.pad = L.kind == kLevelSamples ? 0.5f * L.h + 2e-6f : 2e-6f;
      c->lv.push_back(L);
      tmap += L.nt * L.nt * L.nt;
      pbase += L.npts;
    }
    sd.n_pts = pbase - sd.pt_base;
    for (int k = 0; k < s.m_cap; ++k) kshape[kbase + k] = b;
    kbase += s.m_cap;
    c->sh.push_back(sd);
  }
  hipError_t e = hipMemcpy(D.levels, c->lv.data(), sizeof(LevelDev) * c->lv.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(D.shapes, c->sh.data(), sizeof(ShapeDev) * c->sh.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(D.kshape, kshape.data(), sizeof(int32_t) * kshape.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_fill_i32(D.tile_map, lay.tiles_total, -1, nullptr);
  if (e == hipSuccess) e = launch_fill_f32(D.G, lay.pts_total, 0.f, nullptr);
  if (e == hipSuccess) e = launch_fill_i32(reinterpret_cast<int32_t*>(D.counters), 16, 0, nullptr);
  if (e == hipSuccess) e = launch_fill_i32(reinterpret_cast<int32_t*>(D.tickets), cfg->n_shapes + 1, 0, nullptr);
  if (e == hipSuccess) e = launch_fill_i32(D.tile_cnt, lay.tiles_total + 1, 0, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "erbf_ctx_create");
  }
  *out = c;
  return ERBF_OK;
}

void erbf_ctx_destroy(erbf_ctx* ctx) { delete ctx; }

int erbf_ctx_info(const erbf_ctx* ctx, int32_t* cap_total, int64_t* n_points, int32_t* n_active0) {
  if (!ctx) return fail(ERBF_ERR_INVALID_ARG, "ctx is NULL");
  if (cap_total) *cap_total = ctx->lay.cap_total;
  if (n_points) *n_points = ctx->lay.pts_total;
  if (n_active0) *n_active0 = ctx->sh[0].n_active;
  return ERBF_OK;
}

int erbf_sdf_min(const float* S, int64_t n, float* out_dev, int accumulate, hipStream_t stream) {
  if (!S || !out_dev || n < 1) return fail(ERBF_ERR_INVALID_ARG, "erbf_sdf_min: bad arguments");
  // the ordered-integer key lives in the output word itself
  HIP_TRY(launch_sdf_min(S, n, out_dev, accumulate, reinterpret_cast<int*>(out_dev), stream), "erbf_sdf_min");
  return ERBF_OK;
}

int erbf_targets_from_sdf(const float* S, int64_t n, float m, float* t, hipStream_t stream) {
  if (!S || !t || n < 1) return fail(ERBF_ERR_INVALID_ARG, "erbf_targets_from_sdf: bad arguments");
  if (!(m < 0.f)) return fail(ERBF_ERR_INVALID_ARG, "eq. 3-10 needs a negative minimum signed distance");
  HIP_TRY(launch_targets(S, n, m, t, stream), "erbf_targets_from_sdf");
  return ERBF_OK;
}

int erbf_band_bits(const float* S, int64_t n, float band, uint32_t* bits, hipStream_t stream) {
  if (!S || !bits || n < 1) return fail(ERBF_ERR_INVALID_ARG, "erbf_band_bits: bad arguments");
  HIP_TRY(launch_band_bits(S, n, band, bits, stream), "erbf_band_bits");
  return ERBF_OK;
}

int erbf_octree_bits(const float* S_parent, const uint32_t* parent_bits, int32_t n_parent, uint32_t* child_bits,
                     hipStream_t stream) {
  if (!S_parent || !child_bits || n_parent < 1 || n_parent > 1024)
    return fail(ERBF_ERR_INVALID_ARG, "erbf_octree_bits: bad arguments");
  HIP_TRY(launch_octree_bits(S_parent, parent_bits, n_parent, child_bits, stream), "erbf_octree_bits");
  return ERBF_OK;
}

// A sample level: the samples are binned on the host (a set-up call that
// already synchronises), stably by tile so that each tile's samples keep the
// caller's order; the tiles holding samples become the level's slots in
// ascending tile order, as for a grid level.
static int refine_samples(erbf_ctx* ctx, int32_t shape, ShapeDev& sd, int li, LevelDev& L, const erbf_level* level,
                          hipStream_t stream) {
  const int64_t cap = L.npts, K = level->n_samples;
  if (K < 0 || K > cap) return fail(ERBF_ERR_INVALID_ARG, "n_samples must be in [0, the declared capacity]");
  if (K > 0 && !level->samples) return fail(ERBF_ERR_INVALID_ARG, "samples is NULL");
  DeviceGuard guard(ctx->device);
  Dev& D = ctx->D;
  std::vector<float> xyz((size_t)(3 * K));
  if (K > 0)
    HIP_TRY(hipMemcpy(xyz.data(), level->samples, sizeof(float) * 3 * K, hipMemcpyDeviceToHost), "refine: samples");
  const int n = L.n, nt = L.nt, ntt = nt * nt * nt;
  const double cell = 2.0 / n;
  std::vector<int32_t> tile((size_t)K);
  for (int64_t i = 0; i < K; ++i) {
    int t3[3];
    for (int a = 0; a < 3; ++a) {
      const float v = xyz[3 * i + a];
      if (!(v >= -1.f && v <= 1.f)) return fail(ERBF_ERR_INVALID_ARG, "samples must lie in [-1, 1]^3");
      t3[a] = std::min(n - 1, std::max(0, (int)std::floor(((double)v + 1.0) / cell))) / kTile;
    }
    tile[i] = (t3[2] * nt + t3[1]) * nt + t3[0];
  }
  std::vector<int64_t> order((size_t)K);
  for (int64_t i = 0; i < K; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return tile[a] < tile[b]; });
  std::vector<int32_t> flags(ntt, 0), rank(ntt, -1);
  for (int64_t i = 0; i < K; ++i) flags[tile[i]] = 1;
  int n_act = 0;
  for (int t = 0; t < ntt; ++t)
    if (flags[t]) rank[t] = n_act++;
  std::vector<float4> pos((size_t)std::max<int64_t>(K, 1));
  std::vector<int32_t> start(n_act + 1, 0), sslot((size_t)cap, -1), slots(std::max(n_act, 1));
  for (int64_t k = 0; k < K; ++k) {
    const int64_t i = order[k];
    float4 q;
    q.x = xyz[3 * i];
    q.y = xyz[3 * i + 1];
    q.z = xyz[3 * i + 2];
    int32_t ii = (int32_t)i;
    std::memcpy(&q.w, &ii, sizeof(float));
    pos[k] = q;
    start[rank[tile[i]] + 1] += 1;
    sslot[i] = ctx->slots_used + rank[tile[i]];
  }
  for (int r = 0; r < n_act; ++r) {
    start[r + 1] += start[r];
    slots[r] = ctx->slots_used + r;
  }
  const Layout& lay = ctx->lay;
  if (ctx->samp_used + cap > lay.samp_total || ctx->samp_start_used + ntt + 1 > lay.samp_start_total ||
      D.n_samp_slots + n_act > lay.samp_tiles)
    return fail(ERBF_ERR_STATE, "sample arrays exhausted");
  L.spos = D.samp_pos + ctx->samp_used;
  L.sstart = D.samp_start + ctx->samp_start_used;
  L.sslot = D.samp_slot + ctx->samp_used;
  L.sxyz = level->samples;
  L.n_samples = (int32_t)K;
  L.axis = nullptr;
  L.target = nullptr;
  L.sdf = nullptr;
  L.bits = nullptr;
  if (K > 0)
    HIP_TRY(hipMemcpy(const_cast<float4*>(L.spos), pos.data(), sizeof(float4) * K, hipMemcpyHostToDevice),
            "refine: sample positions");
  HIP_TRY(hipMemcpy(const_cast<int32_t*>(L.sstart), start.data(), sizeof(int32_t) * (n_act + 1),
                    hipMemcpyHostToDevice),
          "refine: sample starts");
  HIP_TRY(hipMemcpy(const_cast<int32_t*>(L.sslot), sslot.data(), sizeof(int32_t) * cap, hipMemcpyHostToDevice),
          "refine: sample slots");
  if (n_act > 0)
    HIP_TRY(hipMemcpy(D.samp_slots + D.n_samp_slots, slots.data(), sizeof(int32_t) * n_act, hipMemcpyHostToDevice),
            "refine: sample slot list");
  HIP_TRY(hipMemcpy(ctx->rflags, flags.data(), sizeof(int32_t) * ntt, hipMemcpyHostToDevice), "refine: flags");
  HIP_TRY(hipMemcpy(&D.levels[li], &L, sizeof(LevelDev), hipMemcpyHostToDevice), "refine: level table");
  HIP_TRY(launch_scan(ctx->rflags, ntt, D.scan_blocks, ctx->rexcl, D.counters + 1, stream), "refine: scan");
  HIP_TRY(launch_tile_assign(D, li, ntt, ctx->rflags, ctx->rexcl, ctx->slots_used, stream), "refine: assign");
  HIP_TRY(launch_fill_f32(D.G + L.pt_base, cap, 0.f, stream), "refine: clear G");
  HIP_TRY(hipStreamSynchronize(stream), "refine: sync");
  L.slot0 = ctx->slots_used;
  L.n_slots = n_act;
  ctx->slots_used += n_act;
  ctx->samp_used += cap;
  ctx->samp_start_used += ntt + 1;
  D.n_samp_slots += n_act;
  sd.n_active += 1;
  if (sd.n_active == 1) sd.slot0 = L.slot0;
  sd.n_slots += L.n_slots;
  HIP_TRY(hipMemcpy(&D.levels[li], &L, sizeof(LevelDev), hipMemcpyHostToDevice), "refine: level table");
  HIP_TRY(hipMemcpy(&D.shapes[shape], &sd, sizeof(ShapeDev), hipMemcpyHostToDevice), "refine: shape table");
  return ERBF_OK;
}

int erbf_refine_level(erbf_ctx* ctx, int32_t shape, const erbf_level* level, hipStream_t stream) {
  if (!ctx || !level) return fail(ERBF_ERR_INVALID_ARG, "ctx and level must be non-NULL");
  if (shape < 0 || shape >= ctx->cfg.n_shapes) return fail(ERBF_ERR_INVALID_ARG, "shape out of range");
  ShapeDev& sd = ctx->sh[shape];
  const erbf_shape_desc& desc = ctx->shape_desc[shape];
  if (sd.n_active >= desc.n_levels) return fail(ERBF_ERR_STATE, "all declared levels already registered");
  const int li = sd.lvl0 + sd.n_active;
  LevelDev& L = ctx->lv[li];
  if (level->n != L.n) return fail(ERBF_ERR_INVALID_ARG, "level n differs from the declared level_n");
  if (L.kind == kLevelSamples) return refine_samples(ctx, shape, sd, li, L, level, stream);
  if (!level->axis) return fail(ERBF_ERR_INVALID_ARG, "level axis is NULL");
  DeviceGuard guard(ctx->device);
  Dev& D = ctx->D;
  {
    // index ranges are computed from the nominal spacing: the table must be
    // the cell-centred grid (to float32 rounding)
    std::vector<float> ax(L.n);
    HIP_TRY(hipMemcpy(ax.data(), level->axis, sizeof(float) * L.n, hipMemcpyDeviceToHost), "refine: axis");
    for (int i = 0; i < L.n; ++i) {
      const double nominal = -1.0 + (2.0 * i + 1.0) / L.n;
      if (!(std::fabs((double)ax[i] - nominal) <= 1e-6))
        return fail(ERBF_ERR_INVALID_ARG, "axis must hold the cell-centred coordinates -1 + (2i+1)/n");
    }
  }
  L.axis = level->axis;
  L.target = level->target;
  L.sdf = level->sdf;
  L.bits = level->active_bits;
  HIP_TRY(hipMemcpy(&D.levels[li], &L, sizeof(LevelDev), hipMemcpyHostToDevice), "refine: level table");
  const int ntt = L.nt * L.nt * L.nt;
  HIP_TRY(launch_tile_flags(D, li, ntt, ctx->rflags, stream), "refine: tile flags");
  HIP_TRY(launch_scan(ctx->rflags, ntt, D.scan_blocks, ctx->rexcl, D.counters + 1, stream), "refine: scan");
  HIP_TRY(launch_tile_assign(D, li, ntt, ctx->rflags, ctx->rexcl, ctx->slots_used, stream), "refine: assign");
  HIP_TRY(launch_fill_f32(D.G + L.pt_base, (int64_t)L.n * L.n * L.n, 0.f, stream), "refine: clear G");
  int64_t n_act = 0;
  HIP_TRY(hipMemcpyAsync(&n_act, D.counters + 1, sizeof(int64_t), hipMemcpyDeviceToHost, stream), "refine: count");
  HIP_TRY(hipStreamSynchronize(stream), "refine: sync");
  L.slot0 = ctx->slots_used;
  L.n_slots = (int32_t)n_act;
  L.dense = n_act == (int64_t)ntt ? 1 : 0;
  ctx->slots_used += (int32_t)n_act;
  sd.n_active += 1;
  if (sd.n_active == 1) sd.slot0 = L.slot0;
  sd.n_slots += L.n_slots;
  HIP_TRY(hipMemcpy(&D.levels[li], &L, sizeof(LevelDev), hipMemcpyHostToDevice), "refine: level table");
  HIP_TRY(hipMemcpy(&D.shapes[shape], &sd, sizeof(ShapeDev), hipMemcpyHostToDevice), "refine: shape table");
  return ERBF_OK;
}

int erbf_eval(erbf_ctx* ctx, const erbf_params* params, float* f_out, erbf_stats* stats_dev, hipStream_t stream) {
  int rc = check_params(ctx, params);
  if (rc) return rc;
  if (!f_out) return fail(ERBF_ERR_INVALID_ARG, "f_out is NULL");
  DeviceGuard guard(ctx->device);
  const Dev& D = ctx->D;
  for (const ShapeDev& s : ctx->sh)
    for (int l = 0; l < s.n_active; ++l) {
      const LevelDev& L = ctx->lv[s.lvl0 + l];
      if (L.bits || L.kind == kLevelSamples) HIP_TRY(launch_fill_f32(f_out + L.pt_base, L.npts, 0.f, stream), "eval: clear");
    }
  HIP_TRY(launch_buckets(D, params->p, params->m_dev, ctx->slots_used, stream), "eval: buckets");
  HIP_TRY(launch_forward(D, ctx->slots_used, false, f_out, 0.f, 0.f, nullptr, stream), "eval: forward");
  if (stats_dev) {
    StatsArgs a{};
    HIP_TRY(launch_stats(D, 0, params->p, params->m_dev, nullptr, stats_dev, a, stream), "eval: stats");
  }
  return ERBF_OK;
}

namespace {
// the loss call; step_inc == nullptr: as erbf_loss_grad.  Otherwise the L2
// gradient stays in grad_out, the weights of eq. 3-21 in the workspace and
// the step counters step_inc are incremented, for the Adam pass of
// erbf_train_step that combines and applies them
int loss_grad_impl(erbf_ctx* ctx, const erbf_params* params, const erbf_loss_cfg* cfg, float* grad_out,
                   erbf_stats* stats_dev, float* f_out, float* G_out, hipStream_t stream, int32_t* step_inc,
                   const int32_t* hold);
}  // namespace

int erbf_loss_grad(erbf_ctx* ctx, const erbf_params* params, const erbf_loss_cfg* cfg, float* grad_out,
                   erbf_stats* stats_dev, float* f_out, float* G_out, hipStream_t stream) {
  return loss_grad_impl(ctx, params, cfg, grad_out, stats_dev, f_out, G_out, stream, nullptr, nullptr);
}

int erbf_train_step(erbf_ctx* ctx, const erbf_params* params, const erbf_loss_cfg* cfg,
                    const erbf_adam_cfg* adam, float* grad_out, float* m1, float* m2, int32_t* step_dev,
                    erbf_stats* stats_dev, float* f_out, float* G_out, hipStream_t stream) {
  if (!adam || !m1 || !m2 || !step_dev) return fail(ERBF_ERR_INVALID_ARG, "erbf_train_step: NULL argument");
  if (!(adam->beta1 >= 0.f && adam->beta1 < 1.f && adam->beta2 >= 0.f && adam->beta2 < 1.f && adam->eps > 0.f))
    return fail(ERBF_ERR_INVALID_ARG, "erbf_train_step: bad Adam hyper-parameters");
  int rc = loss_grad_impl(ctx, params, cfg, grad_out, stats_dev, f_out, G_out, stream, step_dev, adam->hold_dev);
  if (rc) return rc;
  DeviceGuard guard(ctx->device);
  AdamArgs a{adam->lr, adam->lr_dev, adam->beta1, adam->beta2, adam->eps, adam->hold_dev};
  HIP_TRY(launch_adam(ctx->D, params->p, params->m_dev, grad_out, m1, m2, step_dev, a, true, stream), "train: adam");
  return ERBF_OK;
}

namespace {
int loss_grad_impl(erbf_ctx* ctx, const erbf_params* params, const erbf_loss_cfg* cfg, float* grad_out,
                   erbf_stats* stats_dev, float* f_out, float* G_out, hipStream_t stream, int32_t* step_inc,
                   const int32_t* hold) {
  int rc = check_params(ctx, params);
  if (rc) return rc;
  if (!cfg || !grad_out) return fail(ERBF_ERR_INVALID_ARG, "cfg and grad_out must be non-NULL");
  if (cfg->mode < ERBF_MODE_FIXED || cfg->mode > ERBF_MODE_L2) return fail(ERBF_ERR_INVALID_ARG, "unknown mode");
  for (const ShapeDev& s : ctx->sh)
    for (int l = 0; l < s.n_active; ++l)
      if (ctx->lv[s.lvl0 + l].kind == kLevelGrid && !ctx->lv[s.lvl0 + l].target)
        return fail(ERBF_ERR_INVALID_ARG, "a registered grid level has no target");
  DeviceGuard guard(ctx->device);
  const Dev& D = ctx->D;
  if (f_out)
    for (const ShapeDev& s : ctx->sh)
      for (int l = 0; l < s.n_active; ++l) {
        const LevelDev& L = ctx->lv[s.lvl0 + l];
        if (L.bits || L.kind == kLevelSamples)
          HIP_TRY(launch_fill_f32(f_out + L.pt_base, L.npts, 0.f, stream), "loss: clear");
      }
  HIP_TRY(launch_buckets(D, params->p, params->m_dev, ctx->slots_used, stream), "loss: buckets");
  const hipEvent_t* ev = tev_call(ctx);
  const bool fused = (D.variant & kVariantFused) != 0;
  HIP_TRY(launch_forward(D, ctx->slots_used, true, f_out, cfg->tau1, cfg->tau2, ev, stream, fused), "loss: forward");
  uint8_t shared = 0;
  HIP_TRY(launch_backward(D, ctx->slots_used, params->p, D.G, grad_out, ev ? ev + 2 : nullptr, stream, fused,
                          ev && ctx->slots_used > 0 ? ev[1] : nullptr, &shared),
          "loss: backward");
  if (ev) ctx->tshared[ctx->t_used++] = shared;
  StatsArgs a{};
  a.mode = cfg->mode;
  a.lambda = cfg->lambda;
  a.lambda_dev = cfg->lambda_dev;
  a.l1_active = cfg->l1_active;
  a.l1_active_dev = cfg->l1_active_dev;
  a.tau_m = cfg->tau_m;
  a.step_inc = step_inc;
  a.hold = hold;
  HIP_TRY(launch_stats(D, 2, params->p, params->m_dev, grad_out, stats_dev, a, stream, step_inc == nullptr),
          "loss: stats");
  if (G_out)
    HIP_TRY(hipMemcpyAsync(G_out, D.G, sizeof(float) * ctx->lay.pts_total, hipMemcpyDeviceToDevice, stream),
            "loss: copy G");
  return ERBF_OK;
}
}  // namespace

int erbf_loss_grad_batched(erbf_ctx* ctx, const erbf_params* params, const erbf_loss_cfg* cfg, float* grad_out,
                           erbf_stats* stats_dev, float* f_out, float* G_out, hipStream_t stream) {
  // a context's shapes share every launch of the step already; this entry
  // point names that use
  return erbf_loss_grad(ctx, params, cfg, grad_out, stats_dev, f_out, G_out, stream);
}

int erbf_loss_grad_minibatch(erbf_ctx* ctx, const erbf_params* params, const erbf_loss_cfg* cfg, const int64_t* pts,
                         int32_t n_pts, float* grad_out, erbf_stats* stats_dev, float* f_out, hipStream_t stream) {
  int rc = check_params(ctx, params);
  if (rc) return rc;
  if (!cfg || !grad_out) return fail(ERBF_ERR_INVALID_ARG, "cfg and grad_out must be non-NULL");
  if (cfg->mode < ERBF_MODE_FIXED || cfg->mode > ERBF_MODE_L2) return fail(ERBF_ERR_INVALID_ARG, "unknown mode");
  if (n_pts < 0 || n_pts > ctx->D.batch_cap) return fail(ERBF_ERR_INVALID_ARG, "n_pts must be in [0, batch_cap]");
  if (n_pts > 0 && !pts) return fail(ERBF_ERR_INVALID_ARG, "pts must be non-NULL");
  for (const ShapeDev& s : ctx->sh)
    for (int l = 0; l < s.n_active; ++l)
      if (ctx->lv[s.lvl0 + l].kind == kLevelGrid && !ctx->lv[s.lvl0 + l].target)
        return fail(ERBF_ERR_INVALID_ARG, "a registered grid level has no target");
  DeviceGuard guard(ctx->device);
  // bucket lists only for the tiles holding batch points: the other tiles'
  // entries would carry zero moments
  Dev D = ctx->D;
  D.tile_sel = D.sel_buf;
  HIP_TRY(launch_batch_tiles(D, ctx->slots_used, pts, n_pts, D.sel_buf, stream), "batch: tiles");
  // G is zero outside the batch, so the tile backward sees the batch only
  HIP_TRY(launch_fill_f32(D.G, ctx->lay.pts_total, 0.f, stream), "batch: clear G");
  HIP_TRY(launch_buckets(D, params->p, params->m_dev, ctx->slots_used, stream), "batch: buckets");
  StatsArgs a{};
  a.mode = cfg->mode;
  a.lambda = cfg->lambda;
  a.lambda_dev = cfg->lambda_dev;
  a.l1_active = cfg->l1_active;
  a.l1_active_dev = cfg->l1_active_dev;
  a.tau_m = cfg->tau_m;
  HIP_TRY(launch_batch_step(D, ctx->slots_used, pts, n_pts, params->p, params->m_dev, grad_out, f_out, stats_dev,
                            cfg->tau1, cfg->tau2, a, stream),
          "batch: step");
  return ERBF_OK;
}

int erbf_vjp(erbf_ctx* ctx, const erbf_params* params, const float* grad_f, float* grad_out, erbf_stats* stats_dev,
             hipStream_t stream) {
  int rc = check_params(ctx, params);
  if (rc) return rc;
  if (!grad_f || !grad_out) return fail(ERBF_ERR_INVALID_ARG, "grad_f and grad_out must be non-NULL");
  DeviceGuard guard(ctx->device);
  const Dev& D = ctx->D;
  HIP_TRY(launch_buckets(D, params->p, params->m_dev, ctx->slots_used, stream), "vjp: buckets");
  for (const ShapeDev& s : ctx->sh)
    for (int l = 0; l < s.n_active; ++l) {
      const LevelDev& L = ctx->lv[s.lvl0 + l];
      HIP_TRY(launch_mask_copy(D, s.lvl0 + l, L.npts, grad_f, stream), "vjp: mask");
    }
  const hipEvent_t* ev = tev_call(ctx);
  uint8_t shared = 0;
  HIP_TRY(launch_backward(D, ctx->slots_used, params->p, D.G, grad_out, ev ? ev + 2 : nullptr, stream, false,
                          nullptr, &shared),
          "vjp: backward");
  if (ev) {
    // no forward in a VJP: give its pair of events a zero-length interval
    HIP_TRY(hipEventRecord(ev[0], stream), "vjp: event");
    HIP_TRY(hipEventRecord(ev[1], stream), "vjp: event");
    ctx->tshared[ctx->t_used++] = shared;
  }
  if (stats_dev) {
    StatsArgs a{};
    HIP_TRY(launch_stats(D, 1, params->p, params->m_dev, grad_out, stats_dev, a, stream), "vjp: stats");
  }
  return ERBF_OK;
}

int erbf_adam_step(erbf_ctx* ctx, const erbf_params* params, const float* grad, float* m1, float* m2,
                   int32_t* step_dev, const erbf_adam_cfg* cfg, hipStream_t stream) {
  if (!ctx || !params || !params->p || !params->m_dev || !grad || !m1 || !m2 || !step_dev || !cfg)
    return fail(ERBF_ERR_INVALID_ARG, "erbf_adam_step: NULL argument");
  if (!(cfg->beta1 >= 0.f && cfg->beta1 < 1.f && cfg->beta2 >= 0.f && cfg->beta2 < 1.f && cfg->eps > 0.f))
    return fail(ERBF_ERR_INVALID_ARG, "erbf_adam_step: bad hyper-parameters");
  DeviceGuard guard(ctx->device);
  AdamArgs a{cfg->lr, cfg->lr_dev, cfg->beta1, cfg->beta2, cfg->eps, cfg->hold_dev};
  HIP_TRY(launch_adam(ctx->D, params->p, params->m_dev, const_cast<float*>(grad), m1, m2, step_dev, a, false, stream),
          "adam");
  return ERBF_OK;
}

int erbf_set_variant(erbf_ctx* ctx, int32_t variant) {
  if (!ctx || variant < 0 || variant > kVariantAll)
    return fail(ERBF_ERR_INVALID_ARG, "erbf_set_variant: bad arguments");
  ctx->D.variant = variant;
  return ERBF_OK;
}

int erbf_get_variant(const erbf_ctx* ctx, int32_t* variant) {
  if (!ctx || !variant) return fail(ERBF_ERR_INVALID_ARG, "erbf_get_variant: bad arguments");
  *variant = ctx->D.variant;
  return ERBF_OK;
}

namespace {
int max_shape_cap(const erbf_ctx* ctx) {
  int c = 1;
  for (const erbf_shape_desc& d : ctx->shape_desc) c = std::max(c, d.m_cap);
  return c;
}
void apply_launch(erbf_ctx* ctx, const erbf_launch_cfg& c) {
  ctx->D.variant = c.variant;
  ctx->D.slot_chunk = c.slot_chunk;
  ctx->D.samp_split = c.samp_split;
  ctx->D.bucket_rank = c.bucket_rank;
  ctx->D.fwd_chunk = c.fwd_chunk;
  ctx->D.bwd_waves = c.bwd_waves;
  ctx->D.tile_order_on = c.tile_order;
}
erbf_launch_cfg current_launch(const erbf_ctx* ctx) {
  return erbf_launch_cfg{ctx->D.variant,   ctx->D.slot_chunk, ctx->D.samp_split,   ctx->D.bucket_rank,
                         ctx->D.fwd_chunk, ctx->D.bwd_waves,  ctx->D.tile_order_on};
}
int32_t current_field(const erbf_launch_cfg& c, int field) {
  const int32_t f[] = {c.variant, c.slot_chunk, c.samp_split, c.bucket_rank, c.fwd_chunk, c.bwd_waves, c.tile_order};
  return f[field];
}
erbf_launch_cfg with(erbf_launch_cfg c, int field, int32_t v) {
  int32_t* f[] = {&c.variant,   &c.slot_chunk, &c.samp_split, &c.bucket_rank,
                  &c.fwd_chunk, &c.bwd_waves,  &c.tile_order};
  *f[field] = v;
  return c;
}
}  // namespace

int erbf_set_launch(erbf_ctx* ctx, const erbf_launch_cfg* cfg) {
  if (!ctx || !cfg || cfg->variant < 0 || cfg->variant > kVariantAll || cfg->slot_chunk < 0 ||
      cfg->slot_chunk > 256 || cfg->samp_split < 1 || cfg->samp_split > kSampSplitMax ||
      (cfg->bucket_rank != 0 && cfg->bucket_rank != 1) ||
      (cfg->fwd_chunk != 64 && cfg->fwd_chunk != 128 && cfg->fwd_chunk != 256) ||
      (cfg->bwd_waves != 2 && cfg->bwd_waves != 4 && cfg->bwd_waves != 8) ||
      (cfg->tile_order != 0 && cfg->tile_order != 1))
    return fail(ERBF_ERR_INVALID_ARG, "erbf_set_launch: bad arguments");
  if (cfg->bucket_rank && max_shape_cap(ctx) > kRankMaxCap)
    return fail(ERBF_ERR_UNSUPPORTED, "erbf_set_launch: ranked tile lists need shape capacities <= 32768");
  apply_launch(ctx, *cfg);
  return ERBF_OK;
}

int erbf_get_launch(const erbf_ctx* ctx, erbf_launch_cfg* cfg) {
  if (!ctx || !cfg) return fail(ERBF_ERR_INVALID_ARG, "erbf_get_launch: bad arguments");
  *cfg = current_launch(ctx);
  return ERBF_OK;
}

int erbf_autotune(erbf_ctx* ctx, const erbf_params* params, const erbf_loss_cfg* cfg, float* grad_scratch,
                  int32_t reps, int32_t* chosen, float* times_ms, hipStream_t stream) {
  int rc = check_params(ctx, params);
  if (rc) return rc;
  if (!cfg || !grad_scratch || reps < 1) return fail(ERBF_ERR_INVALID_ARG, "erbf_autotune: bad arguments");
  DeviceGuard guard(ctx->device);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence), "autotune: event");
  hipError_t ce = hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
  if (ce != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(ce, "autotune: event");
  }
  const int saved_tmax = ctx->t_max;
  ctx->t_max = 0;  // no per-kernel timing while tuning
  const Dev saved = ctx->D;
  int status = ERBF_OK;
  // mean time of one erbf_loss_grad under the context's current choices
  auto time_it = [&](float* ms_out) -> int {
    int st = erbf_loss_grad(ctx, params, cfg, grad_scratch, nullptr, nullptr, nullptr, stream);  // warm-up
    if (st != ERBF_OK) return st;
    hipError_t e = hipEventRecord(e0, stream);
    for (int r = 0; r < reps && e == hipSuccess && st == ERBF_OK; ++r)
      st = erbf_loss_grad(ctx, params, cfg, grad_scratch, nullptr, nullptr, nullptr, stream);
    if (st != ERBF_OK) return st;
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) return hip_fail(e, "autotune: timing");
    *ms_out = ms / (float)reps;
    return ERBF_OK;
  };
  erbf_launch_cfg best{0, 0, saved.samp_split, saved.bucket_rank, saved.fwd_chunk, saved.bwd_waves,
                       saved.tile_order_on};
  float best_ms = 0.f;
  bool have = false;
  auto consider = [&](const erbf_launch_cfg& c, float* ms_slot) -> int {
    apply_launch(ctx, c);
    float ms = 0.f;
    const int st = time_it(&ms);
    if (st != ERBF_OK) return st;
    if (ms_slot) *ms_slot = ms;
    if (!have || ms < best_ms) {
      best = c;
      best_ms = ms;
      have = true;
    }
    return ERBF_OK;
  };
  // 1. the launch variant
  for (int v = 0; v <= kVariantAll && status == ERBF_OK; ++v) {
    if ((v & kVariantBwdPersistent) && (v & kVariantFused)) {
      // the fused kernel has no separate backward launch: same as v - 2
      if (times_ms) times_ms[v] = -1.f;
      continue;
    }
    status = consider(with(best, 0, v), times_ms ? times_ms + v : nullptr);
  }
  // then one choice at a time, each from the best set so far: (field, the
  // values tried)
  struct Axis {
    int field, n, v[3];
  };
  const Axis axes[] = {
      {1, 3, {2, 8, 32}},     // XCD runs of the grid launches
      {6, 2, {0, 1}},         // tiles longest list first or in slot order
      {5, 3, {2, 4, 8}},      // backward waves per tile
      {4, 3, {64, 128, 256}}, // forward records staged per chunk
      {2, 3, {8, 16, 32}},    // sample tiles' split
      {3, 2, {0, 1}},         // ranked or radix-sorted tile lists
  };
  for (const Axis& a : axes) {
    if (status != ERBF_OK) break;
    if (a.field == 2 && ctx->D.n_samp_slots == 0) continue;
    if (a.field == 3 && max_shape_cap(ctx) > kRankMaxCap) continue;
    // the fused step kernel has its own chunk and waves
    if ((a.field == 4 || a.field == 5) && (best.variant & kVariantFused)) continue;
    const erbf_launch_cfg from = best;
    const int32_t cur = current_field(from, a.field);
    for (int k = 0; k < a.n && status == ERBF_OK; ++k)
      if (a.v[k] != cur) status = consider(with(from, a.field, a.v[k]), nullptr);
  }
  ctx->t_max = saved_tmax;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status == ERBF_OK) {
    apply_launch(ctx, best);
    if (chosen) *chosen = best.variant;
  } else {
    ctx->D.variant = saved.variant;
    ctx->D.slot_chunk = saved.slot_chunk;
    ctx->D.samp_split = saved.samp_split;
    ctx->D.bucket_rank = saved.bucket_rank;
    ctx->D.fwd_chunk = saved.fwd_chunk;
    ctx->D.bwd_waves = saved.bwd_waves;
    ctx->D.tile_order_on = saved.tile_order_on;
  }
  return status;
}

int erbf_timing_enable(erbf_ctx* ctx, int32_t max_calls) {
  if (!ctx || max_calls < 0) return fail(ERBF_ERR_INVALID_ARG, "erbf_timing_enable: bad arguments");
  DeviceGuard guard(ctx->device);
  const size_t need = kEvPerCall * (size_t)max_calls;
  while (ctx->tev.size() < need) {
    hipEvent_t e;
    // timing only: without the system-scope fence, recording an event does
    // not write back and invalidate the caches around the timed kernels
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreate");
    ctx->tev.push_back(e);
  }
  ctx->tshared.assign((size_t)max_calls, 0);
  ctx->t_max = max_calls;
  ctx->t_used = 0;
  return ERBF_OK;
}

int erbf_timing_read(erbf_ctx* ctx, double* ms, int32_t* n_calls) {
  if (!ctx || !ms) return fail(ERBF_ERR_INVALID_ARG, "erbf_timing_read: NULL argument");
  DeviceGuard guard(ctx->device);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < ctx->t_used; ++k) {
    const hipEvent_t* e = &ctx->tev[kEvPerCall * k];
    HIP_TRY(hipEventSynchronize(e[5]), "timing: sync");
    const uint8_t sh = ctx->tshared[k];
    for (int i = 0; i < 3; ++i) {
      // an interval that starts at the previous kernel's stop event
      const hipEvent_t start = (i == 1 && (sh & 1)) ? e[1] : ((i == 2 && (sh & 2)) ? e[3] : e[2 * i]);
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, start, e[2 * i + 1]), "timing: elapsed");
      acc[i] += t;
    }
  }
  for (int i = 0; i < 3; ++i) ms[i] = acc[i];
  if (n_calls) *n_calls = ctx->t_used;
  ctx->t_used = 0;
  return ERBF_OK;
}

namespace {
int check_sched(const erbf_ctx* ctx, const erbf_sched_cfg* cfg, const erbf_sched_state* st) {
  if (!ctx || !cfg || !st) return fail(ERBF_ERR_INVALID_ARG, "ctx, cfg and state must be non-NULL");
  if (cfg->k_l2 < 1 || cfg->k_l2 > 32 || cfg->k_l1 < 1 || cfg->k_l1 > 64)
    return fail(ERBF_ERR_INVALID_ARG, "k_l2 must be in [1, 32] and k_l1 in [1, 64]");
  if (!(cfg->T_e < cfg->M_e) || cfg->T_e < 1) return fail(ERBF_ERR_INVALID_ARG, "need 1 <= T_e < M_e");
  if (!(cfg->tau_d >= 0.f) || !(cfg->lr0 > 0.f) || !(cfg->lr_final > 0.f) || !(cfg->lr_min > 0.f))
    return fail(ERBF_ERR_INVALID_ARG, "tau_d >= 0 and positive learning rates required");
  if (!st->epoch || !st->l1_active || !st->final_phase || !st->add_request || !st->refine_request || !st->b_f ||
      !st->n_pruned || !st->lr || !st->l2_ring || !st->bf_ring)
    return fail(ERBF_ERR_INVALID_ARG, "every control-state array must be non-NULL");
  return ERBF_OK;
}
}  // namespace

int erbf_sched_init(erbf_ctx* ctx, const erbf_sched_cfg* cfg, const erbf_sched_state* state, hipStream_t stream) {
  int rc = check_sched(ctx, cfg, state);
  if (rc) return rc;
  DeviceGuard guard(ctx->device);
  HIP_TRY(launch_sched_init(ctx->D, *state, *cfg, stream), "sched: init");
  return ERBF_OK;
}

int erbf_sched_step(erbf_ctx* ctx, const erbf_params* params, const erbf_sched_cfg* cfg,
                    const erbf_sched_state* state, const erbf_stats* stats_dev, float* m1, float* m2,
                    hipStream_t stream) {
  int rc = check_params(ctx, params);
  if (rc) return rc;
  rc = check_sched(ctx, cfg, state);
  if (rc) return rc;
  if (!stats_dev) return fail(ERBF_ERR_INVALID_ARG, "stats_dev must be non-NULL");
  DeviceGuard guard(ctx->device);
  HIP_TRY(launch_sched_step(ctx->D, params->p, params->p, params->m_dev, m1, m2, *state, *cfg, stats_dev, stream),
          "sched: step");
  return ERBF_OK;
}

int erbf_seed_from_error(erbf_ctx* ctx, const erbf_params* params, int32_t shape, const float* resid,
                         float resid_scale, int64_t n_idall, const erbf_seed_cfg* cfg, float* m1, float* m2,
                         int32_t* n_added, hipStream_t stream) {
  int rc = check_params(ctx, params);
  if (rc) return rc;
  if (!resid || !cfg || !n_added) return fail(ERBF_ERR_INVALID_ARG, "resid, cfg and n_added must be non-NULL");
  *n_added = 0;
  if (shape < 0 || shape >= ctx->cfg.n_shapes) return fail(ERBF_ERR_INVALID_ARG, "shape out of range");
  if (!(cfg->top_frac > 0.f && cfg->top_frac <= 0.05f)) return fail(ERBF_ERR_INVALID_ARG, "top_frac must be in (0, 0.05]");
  if (cfg->k_new < 1 || cfg->k_new > 4096) return fail(ERBF_ERR_INVALID_ARG, "k_new must be in [1, 4096]");
  if (!(cfg->eps > 0.f)) return fail(ERBF_ERR_INVALID_ARG, "eps must be > 0");
  if (!(resid_scale > 0.f)) return fail(ERBF_ERR_INVALID_ARG, "resid_scale must be > 0");
  if (cfg->w_rule != 0 && cfg->w_rule != 1) return fail(ERBF_ERR_INVALID_ARG, "w_rule must be 0 or 1");
  if (n_idall < 0) return fail(ERBF_ERR_INVALID_ARG, "n_idall must be >= 0");
  const ShapeDev& sd = ctx->sh[shape];
  if (sd.n_active < 1) return fail(ERBF_ERR_STATE, "shape has no registered level");
  int64_t npts = 0;
  int finest = -1;
  int samp_levels[ERBF_MAX_LEVELS];
  int64_t samp_counts[ERBF_MAX_LEVELS];
  int n_samp_levels = 0;
  for (int l = 0; l < sd.n_active; ++l) {
    const LevelDev& L = ctx->lv[sd.lvl0 + l];
    npts += L.npts;
    if (L.kind != kLevelGrid) {   // surface samples: neighbours and dbar, never candidates
      samp_levels[n_samp_levels] = sd.lvl0 + l;
      samp_counts[n_samp_levels++] = L.n_samples;
      continue;
    }
    if (!L.sdf) return fail(ERBF_ERR_INVALID_ARG, "seeding needs the raw SDF of every registered grid level");
    if (finest < 0 || L.n > ctx->lv[finest].n) finest = sd.lvl0 + l;
  }
  if (finest < 0) return fail(ERBF_ERR_STATE, "shape has no registered grid level");
  if (npts >= ((int64_t)1 << 32)) return fail(ERBF_ERR_UNSUPPORTED, "seeding supports < 2^32 points per shape");
  const int64_t K = (int64_t)std::ceil((double)cfg->top_frac * (double)n_idall);
  if (K == 0) return ERBF_OK;
  if (K > ctx->D.cand_cap) return fail(ERBF_ERR_WORKSPACE, "candidate list exceeds the workspace");
  DeviceGuard guard(ctx->device);
  const Dev& D = ctx->D;
  // finest spacing from the axis table itself
  float h_fine = 2.0f / (float)ctx->lv[finest].n;
  if (ctx->lv[finest].n > 1) {
    float a2[2];
    HIP_TRY(hipMemcpyAsync(a2, ctx->lv[finest].axis, 2 * sizeof(float), hipMemcpyDeviceToHost, stream), "seed: axis");
    HIP_TRY(hipStreamSynchronize(stream), "seed: sync");
    h_fine = a2[1] - a2[0];
  }
  const float r_nms = cfg->r_nms > 0.f ? cfg->r_nms : 2.0f * h_fine;
  const float floor_abs = std::max(cfg->min_abs_err, cfg->eps);
  HIP_TRY(launch_seed_select(D, shape, npts, resid, resid_scale, floor_abs, r_nms, K, stream), "seed: select");
  int32_t n_cand = 0, n_kept = 0;
  if (seed_misc_counts(D, &n_cand, &n_kept, stream) != 0) return fail(ERBF_ERR_HIP, "seed: reading counts");
  int32_t m_now = 0;
  HIP_TRY(hipMemcpyAsync(&m_now, params->m_dev + shape, sizeof(int32_t), hipMemcpyDeviceToHost, stream), "seed: m");
  HIP_TRY(hipStreamSynchronize(stream), "seed: sync");
  const int n_add = std::min(cfg->k_new, n_kept);
  if (n_add == 0) return ERBF_OK;
  if (m_now < 0 || m_now + n_add > sd.cap)
    return fail(ERBF_ERR_CAPACITY, "seeding " + std::to_string(n_add) + " kernels exceeds the shape capacity");
  HIP_TRY(launch_seed_write(D, shape, n_add, params->p, params->m_dev, resid, resid_scale, m1, m2, cfg->eps,
                            cfg->w_rule, h_fine, samp_levels, samp_counts, n_samp_levels, stream),
          "seed: write");
  HIP_TRY(hipStreamSynchronize(stream), "seed: sync");
  *n_added = n_add;
  return ERBF_OK;
}

int erbf_init_inscribed(erbf_ctx* ctx, const erbf_params* params, int32_t shape, float gamma, int32_t max_centres,
                        float* m1, float* m2, int32_t* n_centres, int64_t* n_left, hipStream_t stream) {
  int rc = check_params(ctx, params);
  if (rc) return rc;
  if (!n_centres || !n_left) return fail(ERBF_ERR_INVALID_ARG, "n_centres and n_left must be non-NULL");
  *n_centres = 0;
  *n_left = 0;
  if (shape < 0 || shape >= ctx->cfg.n_shapes) return fail(ERBF_ERR_INVALID_ARG, "shape out of range");
  if (!(gamma > 0.f && gamma < 1.f)) return fail(ERBF_ERR_INVALID_ARG, "gamma must be in (0, 1)");
  const ShapeDev& sd = ctx->sh[shape];
  if (sd.n_active < 1) return fail(ERBF_ERR_STATE, "shape has no registered level");
  int64_t npts = 0, n_samples = 0;
  for (int l = 0; l < sd.n_active; ++l) {
    const LevelDev& L = ctx->lv[sd.lvl0 + l];
    npts += L.npts;
    if (L.kind != kLevelGrid) {
      n_samples += L.n_samples;
      continue;
    }
    if (!L.sdf || !L.target)
      return fail(ERBF_ERR_INVALID_ARG,
                  "initialisation needs the targets and the raw SDF of every registered grid level");
  }
  if (npts >= (int64_t)UINT32_MAX) return fail(ERBF_ERR_UNSUPPORTED, "initialisation supports < 2^32 - 1 points per shape");
  const int m_max = max_centres <= 0 ? sd.cap : std::min(max_centres, sd.cap);
  DeviceGuard guard(ctx->device);
  const Dev& D = ctx->D;
  HIP_TRY(launch_init_inscribed(D, shape, (uint32_t)npts, n_samples > 0, m_max, sd.cap, gamma, params->p,
                                params->m_dev, m1, m2, stream),
          "init: launch");
  if (init_results(D, n_centres, n_left, stream) != 0) return fail(ERBF_ERR_HIP, "init: reading counts");
  return ERBF_OK;
}

/* ---- surface evaluation (Section 4) ---- */

int erbf_sdf_from_targets(const float* t, int64_t n, float m, float* S, hipStream_t stream) {
  if (!t || !S || n < 1) return fail(ERBF_ERR_INVALID_ARG, "erbf_sdf_from_targets: bad arguments");
  if (!(m < 0.f)) return fail(ERBF_ERR_INVALID_ARG, "eq. 3-10 needs a negative minimum signed distance");
  HIP_TRY(launch_sdf_from_targets(t, n, m, S, stream), "erbf_sdf_from_targets");
  return ERBF_OK;
}

namespace {
struct SurfScratch {
  size_t cnt, off, blocks, total, bytes;
};
SurfScratch surf_scratch(int64_t m3) {
  SurfScratch L{};
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o = align256(o + b); return r; };
  L.cnt = take(sizeof(int32_t) * (size_t)m3);
  L.off = take(sizeof(int32_t) * (size_t)(m3 + 1));
  L.blocks = take(sizeof(int32_t) * (size_t)(m3 / 1024 + 2));
  L.total = take(sizeof(int64_t));
  L.bytes = o;
  return L;
}
}  // namespace

int erbf_surface_scratch_size(int32_t n, size_t* bytes) {
  if (!bytes || n < 2 || n > 1024) return fail(ERBF_ERR_INVALID_ARG, "erbf_surface_scratch_size: n must be in [2, 1024]");
  const int64_t m = n - 1;
  *bytes = surf_scratch(m * m * m).bytes;
  return ERBF_OK;
}

int erbf_surface_extract(const float* F, int32_t n, const float* axis, float iso, void* scratch, size_t scratch_bytes,
                         float* tris, int64_t tri_cap, int64_t* n_tris, hipStream_t stream) {
  if (!F || !axis || !scratch || !n_tris || n < 2 || n > 1024 || tri_cap < 0 || (tri_cap > 0 && !tris))
    return fail(ERBF_ERR_INVALID_ARG, "erbf_surface_extract: bad arguments");
  *n_tris = 0;
  const int64_t m = n - 1, m3 = m * m * m;
  const SurfScratch L = surf_scratch(m3);
  if (scratch_bytes < L.bytes) return fail(ERBF_ERR_WORKSPACE, "erbf_surface_extract: scratch too small");
  char* w = static_cast<char*>(scratch);
  int32_t* cnt = reinterpret_cast<int32_t*>(w + L.cnt);
  int32_t* off = reinterpret_cast<int32_t*>(w + L.off);
  int32_t* blocks = reinterpret_cast<int32_t*>(w + L.blocks);
  int64_t* total = reinterpret_cast<int64_t*>(w + L.total);
  HIP_TRY(launch_fill_i32(reinterpret_cast<int32_t*>(total), 2, 0, stream), "surface: clear");
  HIP_TRY(launch_mt_count(F, axis, n, iso, cnt, total, stream), "surface: count");
  int64_t nt = 0;
  HIP_TRY(hipMemcpyAsync(&nt, total, sizeof(int64_t), hipMemcpyDeviceToHost, stream), "surface: count read");
  HIP_TRY(hipStreamSynchronize(stream), "surface: sync");
  *n_tris = nt;
  // the scan and the per-cube offsets are 32-bit
  if (nt >= (int64_t)INT32_MAX) return fail(ERBF_ERR_UNSUPPORTED, "erbf_surface_extract: more than 2^31 triangles");
  HIP_TRY(launch_scan(cnt, (int)m3, blocks, off, nullptr, stream), "surface: scan");
  if (nt > tri_cap) return fail(ERBF_ERR_CAPACITY, "erbf_surface_extract: " + std::to_string(nt) + " triangles exceed tri_cap");
  if (nt > 0) HIP_TRY(launch_mt_emit(F, axis, n, iso, off, tris, tri_cap, stream), "surface: emit");
  HIP_TRY(hipStreamSynchronize(stream), "surface: sync");
  return ERBF_OK;
}

int erbf_surface_sample(const float* tris, int64_t n_tris, const float* u, int64_t n_samples, double* area_scratch,
                        float* pts, float* normals, int32_t* tri_index, hipStream_t stream) {
  if (!tris || n_tris < 1 || !u || n_samples < 1 || !area_scratch || !pts || !normals)
    return fail(ERBF_ERR_INVALID_ARG, "erbf_surface_sample: bad arguments");
  HIP_TRY(launch_surface_sample(tris, n_tris, u, n_samples, area_scratch, pts, normals, tri_index, stream),
          "erbf_surface_sample");
  return ERBF_OK;
}

int erbf_surface_metrics(const float* Pt, const float* Nt, int64_t nt, const float* Pr, const float* Nr, int64_t nr,
                         double* scratch, double* out, hipStream_t stream) {
  if (!Pt || !Nt || !Pr || !Nr || nt < 1 || nr < 1 || !scratch || !out)
    return fail(ERBF_ERR_INVALID_ARG, "erbf_surface_metrics: bad arguments");
  HIP_TRY(launch_surface_metrics(Pt, Nt, nt, Pr, Nr, nr, scratch, out, stream), "erbf_surface_metrics");
  return ERBF_OK;
}

int erbf_surface_metrics_noalloc(const float* Pt, const float* Nt, int64_t nt, const float* Pr, const float* Nr,
                                 int64_t nr, double* out, hipStream_t stream) {
  if (!Pt || !Nt || !Pr || !Nr || nt < 1 || nr < 1 || !out)
    return fail(ERBF_ERR_INVALID_ARG, "erbf_surface_metrics_noalloc: bad arguments");
  if (nt > kNoallocMetricsPoints - nr)
    return fail(ERBF_ERR_INVALID_ARG, "erbf_surface_metrics_noalloc: nt + nr = " + std::to_string(nt + nr) +
                                          " exceeds the built-in scratch limit of " +
                                          std::to_string(kNoallocMetricsPoints) + " points");
  double* scr = nullptr;
  HIP_TRY(noalloc_metrics_scratch(&scr), "erbf_surface_metrics_noalloc: scratch address");
  HIP_TRY(launch_surface_metrics(Pt, Nt, nt, Pr, Nr, nr, scr, out, stream), "erbf_surface_metrics_noalloc");
  return ERBF_OK;
}

}  // extern "C"
