// Internal device tables and kernel launch declarations of the ERBF library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "erbf.h"

namespace erbf {

constexpr int kOrderClasses = 64;   // list-length classes of the tile launch order
constexpr int kTile = 8;            // grid points per tile edge (tile = 8^3 points)
constexpr int kRecF4 = 3;           // float4 per kernel record
constexpr float kLog2e = 1.4426950408889634f;

// launch variants chosen by the autotuner (bit flags)
constexpr int kVariantFwdPersistent = 1;   // forward tiles walked by a persistent grid
constexpr int kVariantBwdPersistent = 2;   // backward tiles walked by a persistent grid (separate kernels)
constexpr int kVariantFused = 4;           // the loss call's forward and backward tiles in one kernel
constexpr int kVariantAll = 7;

constexpr int kHitCapMax = 512;   // most tile slots the count pass keeps per kernel
constexpr int kSampSplitMax = 32;  // most workgroups per active sample tile (parts of its kernel list)
constexpr int kLevelGrid = 0;      // cell-centred grid of n^3 points
constexpr int kLevelSamples = 1;   // surface samples binned into the tiles of an n^3-cell grid

// Per-level table entry, mirrored on the device.
struct LevelDev {
  int32_t n, nt;            // points (sample levels: binning cells) / tiles per axis
  int32_t shape;            // owning shape
  int32_t slot0;            // first active-tile slot of this level
  int32_t n_slots;          // active tiles
  int32_t tmap0;            // offset of this level's tile map (nt^3 int32)
  int64_t pt_base;          // offset of this level in per-point arrays
  int64_t npts;             // entries in per-point arrays: n^3, or the sample capacity
  float lo, h;              // axis[0] and nominal spacing 2/n (used for index ranges only)
  float pad;                // tile boxes reach this far past their outer points (samples: the
                            // half cell, so the boxes tile space)
  int32_t dense;            // grid levels whose every tile is active: tile t has slot slot0 + t
  int32_t kind;             // kLevelGrid or kLevelSamples
  int32_t n_samples;        // sample levels: samples registered
  const float* axis;
  const float* target;
  const float* sdf;
  const uint32_t* bits;
  const float* sxyz;        // sample levels: the caller's [n_samples * 3] coordinates
  const float4* spos;       // sample levels: samples by tile (x, y, z, original index as int bits)
  const int32_t* sstart;    // sample levels: [n_slots + 1] first spos entry of each active tile
  const int32_t* sslot;     // sample levels: [capacity] tile slot of each sample, -1 if none
};

// Per-shape table entry, mirrored on the device.
struct ShapeDev {
  int32_t kbase, cap;       // kernel slot range
  int32_t lvl0;             // first level-table index
  int32_t n_active;         // active levels
  int32_t slot0, n_slots;   // active-tile slot range over the active levels
  int64_t pt_base, n_pts;   // per-point range over the active levels
};

// Partial statistics of one forward tile.
struct TileStat {
  double l2;
  float max_abs_e;
  int32_t n_idall;
  int64_t p_fwd;           // in-ball pairs at active points of the tile
};


// Slice sums of the step statistics (one per stats block).
constexpr int kStatParts = 64;   // blocks per shape; one wave sums them
struct StatPart {
  double l2, nid, pf, pb, l1, num, den;
  float mx;
  int32_t pad;
};

// Launch plumbing shared by the .hip translation units.
struct Dev {
  // tables
  LevelDev* levels;         // [n_levels_total]
  ShapeDev* shapes;         // [n_shapes]
  int32_t* kshape;          // [cap_total] shape of each kernel slot
  int2* slot_tile;          // [tiles_total] (level index, tile linear id) per active slot
  int32_t* tile_map;        // [tiles_total] slot of each tile or -1
  // buckets
  int32_t* tile_start;      // [tiles_total + 1]
  int32_t* tile_cnt;        // [tiles_total] rank mode: entries of each tile (0 between builds)
  int64_t* tile_start64;    // [tiles_total + 1] rank mode: exclusive scan of tile_cnt
  int32_t* kslot;           // [pair_cap] tile slot of each kernel-major entry (sort input, kept)
  int32_t* kj;              // [pair_cap] kernel of each kernel-major entry
  int32_t* sort_keys[2];    // [pair_cap] radix ping-pong between passes
  int32_t* sort_vals[2];    // [pair_cap]
  int32_t* sort_j[2];       // [pair_cap]
  int32_t* rhist;           // [256 * radix_nb + 1] digit counts per sort block
  int32_t* rhist_ex;        // [256 * radix_nb + 256] prefix within each digit's row, then row totals
  int32_t* tile_keys;       // [pair_cap] tile slot of each tile-major entry (sorted)
  int32_t* tile_e;          // [pair_cap] kernel-major index of each tile-major entry
  int32_t* items;           // [pair_cap] kernel of each tile-major entry: ascending within a tile
  int32_t* tile_order;      // [tiles_total] active slots, longest list first (launch order of the tile kernels)
  int32_t* order_hist;      // [kOrderClasses * (tiles_total / 256 + 2)] list-length classes of each block of 256 slots
  int32_t* kcnt;            // [cap_total + 1] bucket entries of each kernel
  int32_t* hits;            // [cap_total * hit_cap] tile slots a kernel hits, in visit order (count pass)
  int64_t* kstart;          // [cap_total + 1] exclusive scan of kcnt
  int32_t* kblock;          // [cap_total / 4 + 1] kcnt summed over each count block (four kernels)
  int64_t* kblock_ex;       // [cap_total / 4 + 2] exclusive scan of kblock
  float2* partials;         // [5 * pair_cap] the 10 backward moments of each entry, kernel-major
  int32_t* sel_buf;         // [tiles_total] scratch of the tile selection below
  const int32_t* tile_sel;  // null, or [tiles_total]: bucket lists only for slots with a non-zero entry
  int32_t* scan_blocks;     // [scan block sums] (int64 when a 64-bit scan uses it)
  // per step
  float4* rec;              // [3 * cap_total]
  float* G;                 // [pts_total]
  TileStat* tstat;          // [tiles_total]
  int64_t* tile_pbwd;       // [tiles_total] in-ball pairs at non-zero-G points of each tile
  int64_t* counters;        // [8]: 0 bucket entries, 1 refine count
  uint32_t* tickets;        // [n_shapes + 1] last-block tickets of the statistics, per shape (0 between calls)
  StatPart* stat_part;      // [n_shapes * kStatParts]
  int32_t* prune_flag;      // [n_shapes] eq. 3-27 due after this step (training control)
  int32_t* sched_held;      // [n_shapes] the control call finds its hold word set (control scratch)
  // mini-batch records, one per batch point (batch order)
  double* b_l2;             // [batch_cap] E^2
  float* b_abs;             // [batch_cap] |E|
  int32_t* b_id;            // [batch_cap] point in id_all
  int32_t* b_pf;            // [batch_cap] in-ball pairs at the point
  int32_t* b_shape;         // [batch_cap] shape of the point, -1 if not a training point
  double2* stat_ab;         // [n_shapes] alpha, beta of eq. 3-21 for the last loss call
  // seeding scratch
  uint32_t* seed_hist;      // [65536]
  int64_t* seed_cand;       // [cand_cap]
  int64_t* seed_keep;       // [cand_cap]
  int32_t* seed_misc;       // [64]
  // sample levels
  float4* samp_pos;         // [total sample capacity]
  int32_t* samp_start;      // [sum over sample levels of tiles + 1]
  int32_t* samp_slot;       // [total sample capacity]
  int32_t* samp_slots;      // [sample-level tiles] slots of every active sample tile
  int32_t n_samp_slots;     // entries of samp_slots in use
  float* samp_f;            // [total sample capacity * kSampSplitMax] forward sum of each (sample, list part)
  int32_t* samp_c;          // [total sample capacity * kSampSplitMax] its in-ball pair count
  int64_t* samp_pb;         // [sample-level tiles * kSampSplitMax] backward pair counts of each list part
  // inscribed-sphere initialisation scratch: nearest-sample squared
  // distances (double, init_cand_cap), candidate mask (init_words), two
  // candidate lists (init_cand_cap each) and 8 result words
  uint32_t* init_scratch;   // [4 * init_cand_cap + init_words + 8]
  int64_t init_words;       // pts_total / 32 + 1
  int64_t init_cand_cap;    // points of the largest shape (all its levels)
  int64_t cand_cap;
  int64_t pair_cap;
  int32_t cap_total;
  int32_t tiles_total;
  int32_t n_shapes;
  float cull_k;
  int32_t weight_map;
  int32_t orientation;      // ERBF_ORIENT_*
  int32_t variant;          // kVariant* flags
  int32_t slot_chunk;       // tile runs per XCD of the grid launches (0: workgroup b takes slot b)
  int32_t samp_split;       // parts of each sample tile's kernel list (workgroups), 1 .. kSampSplitMax
  int32_t bucket_rank;      // 1: tile lists by atomic placement and per-tile ranks; 0: by the radix sort
  int32_t fwd_chunk;        // kernel records a forward tile workgroup stages at a time: 64, 128 or 256
  int32_t bwd_waves;        // waves of a backward tile workgroup: 2, 4 or 8
  int32_t tile_order_on;    // 1: tile kernels take the slots of tile_order (longest list first)
  int32_t packed_keys;      // 1: the sort's keys carry the kernel id in their low 16 bits (slot << 16 | j)
  int32_t rank_words;       // bitmap words per wave of the rank pass (largest shape capacity / 32)
  int32_t persistent_wgs;   // grid of the persistent variants
  int32_t radix_nb;         // blocks of each radix-sort pass
  int32_t hit_cap;          // columns of hits (0: none kept)
  int32_t n_levels_total;   // entries of `levels` (ordered by pt_base)
  int32_t batch_cap;        // largest mini-batch
};

}  // namespace erbf
