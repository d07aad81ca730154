// Host-side launchers of the gfx950 kernels (one translation unit per step).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc {

typedef uint32_t u32;
typedef uint64_t u64;

// Control block of the level-synchronous BFS (device memory, zero-initialised).
struct BfsCtl {
  u32 qlen[2];      // frontier queue lengths, indexed by level parity
  u32 mode;         // expansion mode of the next level: 0 top-down, 1 bottom-up
  u32 done;         // set once a level produced an empty frontier
  u32 depth;        // largest level assigned so far
  u32 blocks_done;  // last-block detection
  u32 bu_levels;    // levels expanded bottom-up
  u32 num_roots;    // components (roots = smallest ID of each component)
  u32 bqlen[2];     // lengths of the queues of big frontier vertices, by level parity
  u64 mu;           // sum of degrees of vertices not yet visited
};

// Intersection classes by degree of the staged endpoint x.
struct IsectParams {
  u32 lane_max;    // d(x) <= lane_max        : lane-per-cover-edge merge
  u32 wave_max;    // d(x) <= wave_max        : wavefront per x, LDS hash
  u32 chunk;       // block items stage N(x) in chunks of at most `chunk` entries
  u32 seg;         // partners per block item
};

// The thresholds in force (set by tc_set_isect_params).
IsectParams current_isect_params();

// Planning output (device), read back once by the host.
struct Plan {
  u32 num_lane_x;   // vertices of the lane class
  u32 num_wave_x;   // vertices of the wavefront class
  u32 num_block_x;  // vertices of the block class
  u32 num_items;    // block work items
  u32 num_cover;    // cover edges |S| = sum of hcnt
  u32 next_wave;    // dynamic work counters
  u32 next_item;
  u32 num_long;     // rows split by a whole workgroup, and their work counter
  u32 next_long;
  u32 bad_records;  // vertices whose record cursor disagrees with hcnt (broken contract)
  u32 hub_lim;      // degree class from which a vertex is a hub (0: no hubs)
  u32 num_hubs;     // hubs, indexed 0 .. num_hubs - 1 in hublist
  u32 num_hub_items;  // work items of the hub pass
};

// ---- hubs -------------------------------------------------------------------------
// The cover edges staged under the highest-degree vertices (hubs) are counted by one
// pass per partner y instead of one intersection per edge: y's pruned list N'(y) (its
// other-level neighbours and its same-level neighbours above y) is streamed once, and
// each entry w looks up the hub bitmask of w (bit k: w is in hub k's pruned list S(h_k))
// against the mask H(y) of the hubs that stage y.  The hubs are the vertices of the top
// degree classes, as many whole classes as fit in max_hubs, from class min_class up.
struct HubParams {
  u32 max_hubs;   // 0 (no hub pass) .. kMaxHubs
  u32 min_class;  // smallest degree class a hub may have
};
constexpr u32 kMaxHubs = 256;
constexpr u32 kHubWords = kMaxHubs / 32;  // words of H(y) per vertex
constexpr u32 kHubChunk = 1024;           // entries of N'(y) per hub work item
constexpr u32 kHubFlag = 0x80000000u;     // hcnt flag of a hub row (its edges go to the hub pass)

// What the split needs for the hub pass.  lim: device word with the hub class
// threshold (0: no hubs, then nothing else is read); hubidx: hub index per hub vertex;
// hy: kHubWords words per vertex, written for the rows that have hub partners; items:
// (y, offset into N'(y)) work items, at most cap, counted in *num_items.
struct HubView {
  const u32* lim;
  const uint8_t* hubidx;
  u32* hy;
  uint2* items;
  u32* num_items;
  u32 cap;
};

struct Item {
  u32 x, seg;  // staged vertex, segment of its partner list
};

// ---- prep ----
void launch_tile_rows(const u32* rowptr, u32 n, u32 m, u32* tile_row, hipStream_t s);
// Component roots: parent[v] = smallest vertex ID of v's component (sampled union-find).
// `mode` is two device words of scratch.
void launch_cc(const u32* rowptr, const u32* colidx, u32 n, u32 m, u32* parent, u32* mode,
               hipStream_t s);
// The first search's roots: mode[0] = v0, the smallest vertex with neighbours (kInf if
// none), parent[v] = v for v0 and the isolated vertices, v0 for the others; mode[2] = 0.
// `mode` is four device words.
void launch_first_root(const u32* rowptr, u32 n, u32* parent, u32* mode, hipStream_t s);
// After the first search: the unreached vertices become their own parents, counted in
// mode[2].
void launch_rest_init(const u32* level, u32 n, u32* parent, u32* mode, hipStream_t s);
// Roots of the unreached vertices: their edges joined (mode[0] = v0 marks the reached
// component), then every parent compressed to its root.
void launch_rest_links(const u32* rowptr, const u32* colidx, u32 n, u32* parent, u32* mode,
                       hipStream_t s);
// vinfo[v] = (L(v) mod 2) << 7 | degree class; hcur[v] = rowptr[v] (the record cursors).
// class_hist (128 words, zeroed; may be null): vertices per degree class, for the
// classes >= hist_min (the others stay 0).
// level = nullptr: every vertex gets parity 0 (all on one level).
void launch_vinfo(const u32* rowptr, const u32* level, u32 n, uint8_t* vinfo, u32* hcur,
                  u32* class_hist, u32 hist_min, hipStream_t s);
// Exclusive scan of in[0..count) into out[0..count] (out[count] = total); in may == out.
// tmp needs scan_tmp_words(count) words.
size_t scan_tmp_words(u32 count);
void launch_scan(const u32* in, u32* out, u32 count, u32* tmp, hipStream_t s);
void launch_validate(const u32* rowptr, const u32* colidx, const u32* tile_row, u32 n, u32 m,
                     u32* flag, hipStream_t s);
// Bounds check of an untrusted CSR on the device: rowptr[0] = 0, non-decreasing,
// rowptr[n] = m, every ID < n.  flag: one device word of scratch.  Synchronises s.
// Returns 0 (valid), -4 (a bound is broken) or -3 (a HIP call failed).
int check_csr_bounds(const u32* rowptr, const u32* colidx, u32 n, u32 m, u32* flag,
                     hipStream_t s);
bool validate_rowptr_ok(const u32* rowptr, u32 n, u32 m, u32* flag, hipStream_t s);

// ---- BFS ----
// queue0 / queue1: n words each; bigq0 / bigq1: bfs_big_cap(n, m) words each (room for
// every vertex whose list is shared by the grid in top-down levels).
// keep: vertices with a level from an earlier search keep it and take no part (level
// holds that search's result; the others must be kInf).
void launch_bfs_init(const u32* rowptr, const u32* parent, u32 n, u32* level, u32* queue0,
                     u32* bigq0, u32* fb, BfsCtl* ctl, hipStream_t s, bool keep = false);
// fb: three frontier bitmaps of (n + 31) / 32 words each, zeroed before launch_bfs_init.
// part: bfs_part_words() words of per-workgroup totals; grid <= bfs_grid(n).
void launch_bfs_level(const u32* rowptr, const u32* colidx, u32 n, u32 k, u32* level,
                      u32* queue0, u32* queue1, u32* bigq0, u32* bigq1, u32* fb, BfsCtl* ctl,
                      u64* part, u32 grid, hipStream_t s);
u32 bfs_grid(u32 n);
size_t bfs_part_words();
size_t bfs_big_cap(u32 n, u64 m);
// Persistent top-down levels from level k0 (one cooperative launch, at most max_levels
// levels): run_state is bfs_run_bytes() of device memory (cleared here), grid at most
// bfs_run_grid(n).  False if the launch was refused (the caller then stays with
// launch_bfs_level).  Afterwards the search resumes at level bfs_run_next_level(host copy
// of run_state), with ctl updated; launch_bfs_bitmap rebuilds the frontier bitmaps for
// that level before any launch_bfs_level.
constexpr size_t kBfsRunMaxBytes = 256;  // bfs_run_bytes() is at most this
size_t bfs_run_bytes();
u32 bfs_run_grid(u32 n);
bool launch_bfs_run(const u32* rowptr, const u32* colidx, u32 n, u32 k0, u32 max_levels,
                    u32* level, u32* queue0, u32* queue1, u32* bigq0, u32* bigq1, BfsCtl* ctl,
                    void* run_state, u32 grid, hipStream_t s);
u32 bfs_run_next_level(const void* run_state);
void launch_bfs_bitmap(u32 n, u32 k, const u32* queue0, const u32* queue1, const BfsCtl* ctl,
                       u32* fb, hipStream_t s);

// ---- cover-edge extraction ----
// Per vertex v: colidx2[rowptr[v] .. split[v]) = neighbours on v's level (ascending),
// colidx2[split[v] .. rowptr[v + 1]) = the others (ascending), sabove[v] = the first of
// the former above v, hcnt[v] = |H+(v)|, and the partner records of H+(v) at
// hrec[rowptr[v] .. rowptr[v] + hcnt[v]) (absolute offsets into colidx2; .w = partner).
// colidx2 and hrec hold m entries; hcur comes from launch_vinfo.  long_rows: n words of
// scratch; counters: two words, zeroed before the launch.
// Hub rows get hcnt[v] = |H+(v)| | kHubFlag and no records; a partner that is a hub
// advances its cursor but its record is replaced by a bit of H(y) in hv.hy.
void launch_split_rows(const u32* rowptr, const u32* colidx, const uint8_t* vinfo, u32 n, u32 m,
                       u32* colidx2, u32* split, u32* sabove, u32* hcnt, u32* hcur, uint4* hrec,
                       u32* long_rows, u32* counters, const HubView& hv, hipStream_t s);
// Also counts in plan->bad_records the vertices with hcur[v] != rowptr[v] + |H+(v)|.
void launch_plan(const u32* rowptr, const u32* hcnt, const u32* hcur, u32 n, IsectParams p,
                 u32* lane_x, u32* wave_x, u32* block_x, u32* block_items, Plan* plan,
                 hipStream_t s);
void launch_fill_items(const u32* rowptr, const u32* hcnt, const u32* block_x,
                       const u32* item_off, u32 nbx, IsectParams p, Item* items,
                       hipStream_t s);

// ---- hub pass ----
// Picks the hub class threshold from class_hist (plan->hub_lim) and numbers the hubs
// (hubidx, hublist, plan->num_hubs).
void launch_hub_select(const uint8_t* vinfo, u32 n, const u32* class_hist, HubParams hp,
                       uint8_t* hubidx, u32* hublist, Plan* plan, hipStream_t s);
// Words of the window cut table and of the hub bitmasks (per vertex) for nhubs hubs.
size_t hub_cut_words(u32 nhubs, u32 n);
u32 hub_mask_words(u32 nhubs);
// Builds the hub bitmasks of all n vertices (hub_mask_words(nhubs) words each; the
// window kernel takes about 70 KB of LDS per workgroup).
void launch_hub_masks(const u32* rowptr, const u32* colidx2, const u32* split,
                      const u32* sabove, const u32* hublist, u32 nhubs, u32 n, u32* cuts,
                      u32* hubmask, hipStream_t s);
// Counts the hub items' triangles into the c1 counter (no LDS); with split_stats the
// same-level apexes go to the t2 counter instead.  With tri (device, per-vertex counts)
// each triangle {h, y, w} also adds 1 to t(h), t(y) and t(w); hublist maps hub numbers
// to vertex IDs.
void launch_hub_count(const u32* rowptr, const u32* colidx2, const u32* sabove,
                      const u32* split, u32 nhubs, const u32* hy, const u32* hubmask,
                      const uint2* items, u32 nitems, u64* ctr, bool split_stats,
                      const u32* hublist, u64* tri, hipStream_t s);

// ---- intersection ----
// The intersection launchers take the split's outputs in one struct.  pruned: count
// only T (in the c1 and t2 slots), from the level-split rows (colidx2 holds m entries
// plus 4 readable padding entries) and the partner records; otherwise c1, c2 and t2 from
// colidx, with the partners read from the records' .w fields.  split_stats (with
// pruned): every same-level apex is tallied in t2 and every other-level one in c1.
struct SplitView {
  const u32* colidx2;
  const u32* split;
  const u32* sabove;
  const u32* hcnt;
  const uint4* hrec;
  const u32* tail4b;
};
void launch_isect_lane(const u32* rowptr, const u32* colidx, const uint8_t* vinfo,
                       const SplitView& sv, const u32* lane_x, u32 nlx, u64* ctr, u64* tri,
                       hipStream_t s);
void launch_isect_wave(const u32* rowptr, const u32* colidx, u32 m, const u32* tail4,
                       const uint8_t* vinfo, const SplitView& sv, const u32* wave_x, u32 nwx,
                       Plan* plan, u64* ctr, u64* tri, bool pruned, bool split_stats,
                       hipStream_t s);
void launch_tail4(const u32* colidx, u32 m, u32* tail4, hipStream_t s);
void launch_isect_block(const u32* rowptr, const u32* colidx, u32 m, const u32* tail4,
                        const uint8_t* vinfo, const SplitView& sv, const Item* items,
                        u32 nitems, IsectParams p, Plan* plan, u64* ctr, u64* tri, bool pruned,
                        bool split_stats, hipStream_t s);
void launch_finalize(const u64* ctr, u64* out, hipStream_t s);

// ---- batched, fused per-graph pipeline ----
size_t batch_workspace_bytes(u32 num_graphs, u64 total_rows, u64 total_cols);
void launch_batch(const u32* rowptr_cat, const u32* colidx_cat, const int64_t* row_off,
                  const int64_t* col_off, u32 num_graphs, u64 total_rows, u64 total_cols,
                  void* ws, IsectParams p, u64* counts, hipStream_t s);

int num_cus();

}  // namespace tc
