// plan.h -- the histogram handle and the fill plans chosen for it.
#pragma once

#include "../../include/hist.h"
#include "kernels.h"

#include <atomic>
#include <map>
#include <string>
#include <tuple>
#include <vector>

namespace hg {

constexpr int kMaxSegments = 1024;
// Events per chunk of hist_fill_host when the caller passes 0.
constexpr int64_t kHostChunkDefault = (int64_t)1 << 22;

struct HostStreamer;
void host_streamer_destroy(HostStreamer *hs);

// How one fill is launched.
struct Plan {
    int strategy = HIST_STRAT_LDS;   // hist_strategy (never AUTO here)
    int acc = ACC_U32;               // Acc
    int threads = 1024;
    int blocks = 1;
    int copies = 1;
    int32_t win_lo = 0;              // LDS: first bin of the window
    int32_t win_len = 0;             // LDS: window bins (0 = global only); TILED: tile bins
    int merge = MERGE_ATOMIC;
    int64_t per_block = 0;
    int epoch_iters = 1;
    int lds_base = 0;                // bytes before the window (statistics, models, cache)
    int lds = 0;                     // dynamic LDS bytes per workgroup
    int lds_cache = -1;              // out-of-window hot-bin cache offset, -1: none
    int cache_slots = 0;
    int bucket_bits = 0;             // PART: log2 of the bucket width in bins
    int unroll = 0;                  // events per thread and iteration of the fill kernel
    bool shape = false;              // launch through the shape variants (fill_shape.hip)
    int stats_ept = 0;               // 0: statistics fused; else separate kernels, this many
                                     // events per thread
};

// Choices the autotuner (or a test) fixes for a shape; 0 / -1 mean "heuristic".
struct PlanChoice {
    int strategy = HIST_STRAT_AUTO;
    int blocks = 0;          // total workgroups (x-dimension for tiles)
    int blocks_per_cu = 0;
    int copies = 0;
    int merge = -1;
    int64_t win_lo = -1;
    int threads = 0;         // threads per workgroup (0: heuristic)
    int bucket_bits = 0;     // PART: log2 bucket width (0: heuristic)
    int unroll = 0;          // events per thread (0: heuristic; 1, 2, 4, 8 where a variant exists)
    int stats_ept = 0;       // 0: fused statistics; 1, 4, 16: separate reduction kernels
};

}  // namespace hg

struct hist_s {
    int dims = 0;
    uint32_t flags = 0;
    int device = 0;
    int64_t T = 0;
    int S = 0;
    int num_cu = 256;
    int lds_max = 65536;
    hg::AxisDev ax[hg::kMaxDims];
    bool variable[hg::kMaxDims] = {false, false, false};
    std::vector<double> edges_host[hg::kMaxDims];
    double *d_edges[hg::kMaxDims] = {nullptr, nullptr, nullptr};
    hg::ModelSeg *d_model[hg::kMaxDims] = {nullptr, nullptr, nullptr};
    bool trained[hg::kMaxDims] = {false, false, false};
    int index_feature[hg::kMaxDims] = {0, 0, 0};
    double index_mean_window[hg::kMaxDims] = {0, 0, 0};
    double index_max_window[hg::kMaxDims] = {0, 0, 0};
    bool index_narrow[hg::kMaxDims] = {false, false, false};   // at most two candidate bins
    uint64_t *d_cnt = nullptr;
    double *d_sumw = nullptr, *d_sumw2 = nullptr, *d_stats = nullptr;
    void *d_stage = nullptr;
    size_t stage_bytes = 0;
    int32_t *d_gbins = nullptr;
    int64_t gbins_cap = 0;
    void *d_part = nullptr;                              // PART scratch
    size_t part_bytes = 0;
    // PART bucket totals known to be zero (the scatter pass clears them):
    // where they are and how many
    const void *part_zero_at = nullptr;
    int part_zero_n = 0;
    uint64_t *d_entries = nullptr;                       // entry count, inside d_stats' allocation
    hg::PlanChoice forced;                               // hist_set_strategy
    // kernel timing (hist_timing): event pairs around the fill and merge kernels
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, int>> ev_fill, ev_merge;  // indices into ev_pool
    int ev_next = 0;
    std::map<std::tuple<int, int, int>, hg::PlanChoice> tuned;  // (acc, f32, n bucket)
    hg::HostStreamer *host = nullptr;                    // hist_fill_host buffers and copy stream
    // live batches and multi-fill sets that write into this handle's sums:
    // hist_destroy refuses the handle while any holds it
    std::atomic<int> users{0};
};

namespace hg {

hist_status set_error(hist_status st, const char *fmt, ...);
uint64_t host_order_key(double x);
hist_status zero_state(hist_s *h, hipStream_t s);
hist_status ensure_stage(hist_s *h, size_t bytes, hipStream_t s, bool reserving = false);
hist_status ensure_gbins(hist_s *h, int64_t count, hipStream_t s, bool reserving = false);
// The scratch of the plan for fills of up to n_max events (hist_reserve
// without its synchronization).
hist_status reserve_scratch(hist_s *h, int64_t n_max, hist_dtype dtype, bool weighted, hipStream_t s);
FillArgs base_args(const hist_s *h, const void *const *coords, const void *w, int64_t n);
// Places the learned models of the axes in LDS after the statistics area;
// returns the first free LDS byte.
int apply_model_offsets(const hist_s *h, FillArgs &a);
// LDS offsets of the learned models and staged edges of dims axes from byte
// `off` on; returns the first free byte (16-aligned).
int lds_axis_layout(int dims, AxisDev *ax, int off);
Plan make_plan(const hist_s *h, int64_t n, hist_dtype dtype, bool weighted);
// The plan choice hist_tune stored for this handle or its shape, if any.
bool tuned_choice(const hist_s *h, bool weighted, bool f32, PlanChoice &out);
Plan plan_from_choice(const hist_s *h, int64_t n, hist_dtype dtype, bool weighted,
                      const PlanChoice &c);
int timing_event(hist_s *h);
// A fixed device region that replaces a fill's scratch (hist_fill_static):
// the staging slots, or the bin array and partition tables of chunks sized to
// fit it.
struct FixedScratch {
    char *base;
    size_t bytes;
};
hist_status run_plan(hist_s *h, const Plan &p, const void *const *coords, const void *w,
                     int64_t n, hist_dtype dtype, hipStream_t s, const FixedScratch *fx = nullptr);
size_t stage_bytes_for(const Plan &p);
int64_t stage_stride_for(const Plan &p);
int64_t stage_stride_of(int acc, int64_t win_len);   // units of one staging slot
int64_t tiled_chunk(const hist_s *h);
int64_t part_chunk(const hist_s *h);
// Smallest and largest log2 bucket width a PART plan can use (lo > hi: none).
void part_bits_range(const hist_s *h, bool weighted, int lds_base, int &lo, int &hi);
int unroll_of(const hist_s *h, bool f32, bool weighted, int acc);

}  // namespace hg
