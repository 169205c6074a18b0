// Stage machinery shared by batch plans and the server: device buffers of
// one batch of jobs, the job tables, the enqueue of the stage sequence and
// the decoding of per-job results.
#pragma once

#include "common.hpp"

#include <vector>

namespace hra {
// Entries past the N directions of a direction table that stay readable
// (hemisphere tables from dir_table, the allocation-free table):
// k_dirstats prefetches the next 64 entries without clamping, up to 127
// entries past N.
constexpr int DIR_TABLE_PAD = 128;
struct DirTotals;
// Directional statistics of n samples (k_dirstats); with `hist`, the
// direction histogram too, formed from per-block slices in `slices`
// (HIST_BINS words per block; NULL: stream-ordered allocation for the
// launch); at most max_blocks blocks.
hipError_t launch_dirstats(hra_ctx *ctx, const float *normal, int64_t n, const float4 *table, int32_t N,
                           const uint32_t *bits, const hra_dirstats &out, double *c64, uint32_t *cnt, bool hist,
                           hipStream_t s, uint32_t *slices = nullptr, int64_t max_blocks = INT64_MAX);
void classify_from_device_totals(const void *host_totals, int64_t n, int32_t n_dirs, const hra_thresholds *th,
                                 hra_class_report *out);
hipError_t launch_part_totals_raw(const int8_t *axis, const uint32_t *cnt, const double *c64, const int64_t *d_base,
                                  const int64_t *d_count, int n_parts, void *tot, hipStream_t s);
size_t dir_totals_size();
hipError_t launch_setups_raw(const void *d_jobs, int n_jobs, int64_t n_total, const float *point, const int32_t *tri,
                             const uint32_t *axes_bits, unsigned long long *cc, uint32_t *hist, uint32_t *err,
                             hipStream_t s);
size_t setup_job_size();
void fill_setup_job(void *dst, const hra_bvh *bvh, int32_t part, int64_t sample_base, int64_t n, double tool);
void solve_setups(const uint32_t *hist, int32_t *min_count, int32_t *min_mask, int32_t *g_count, int32_t *g_mask);

// Device buffers of one batch of jobs, carved from one allocation.
struct StageBufs {
    float *pt, *nr, *org;
    int32_t *tri;
    uint32_t *bits, *abits;
    float *mean, *absm, *conc;
    int8_t *axis;
    double *c64;
    uint32_t *cnt;
    void *tot;
    unsigned long long *cc;
    uint32_t *chist;
    int64_t *dbase, *dcount;
    SampleJob *dsj;
    CastJob *dcj, *daj;
    void *dsetj;
    // the spatial order of the samples for the hemisphere cast: keys and
    // values twice, and the sort's workspace
    uint64_t *okey0, *okey1;
    uint32_t *oval0, *oval1, *osort;
};

// Shape of one batch: jobs, samples, work items and launch shape.
struct StageShape {
    int32_t n_jobs;
    int64_t S, items, aitems;
    int32_t N, W, rpw, stack, trav, group;
    const float4 *t_hemi, *t_ax;
    SampleJob sj0;
    CastJob cj0, aj0;
};

// Host job tables of a batch: job j is part `part[j]` of hierarchy
// `bvh[j]`, with its samples at rows [base[j], base[j] + count[j]).
struct HostJobs {
    std::vector<int64_t> base, count;
    std::vector<SampleJob> sj;
    std::vector<CastJob> cj, aj;
    std::vector<char> setj;
};

size_t carve_stage(char *base, int64_t S, int32_t W, int32_t n_jobs, StageBufs *out);
void fill_jobs(const StageBufs &B, const std::vector<const hra_bvh *> &bvh, const std::vector<int32_t> &part,
               const std::vector<int64_t> &count, const std::vector<uint64_t> &seed, const std::vector<double> &tool,
               float frac, StageShape *sh, HostJobs *H);
// Bytes of the job tables of n jobs, and their packing into one host block
// laid out like the device tables (dbase, dcount, dsj, dcj, daj, dsetj).
size_t job_table_bytes(int32_t n_jobs);
void pack_jobs(const HostJobs &H, char *dst);
// Copies of a packed job block to the device tables.
hipError_t upload_packed_jobs(const StageBufs &B, const char *src, int32_t n_jobs, hipStream_t s);
// The stage sequence on s.  With a side stream (and its fork and join
// events), the six-axis cast and the setups, which need only the samples
// and the hierarchy, run on it beside the hemisphere cast and the
// statistics, and s waits for them before the copies; without one they
// follow the statistics on s.
hipError_t enqueue_stages(hra_ctx *ctx, const StageShape &sh, const StageBufs &B, void *h_tot,
                          unsigned long long *h_cc, uint32_t *h_ch, hipStream_t s, hipEvent_t *ev, uint32_t *err,
                          hipStream_t side = nullptr, hipEvent_t fork = nullptr, hipEvent_t join = nullptr);
void decode_results(const StageShape &sh, const std::vector<int64_t> &count, const void *h_tot,
                    const unsigned long long *h_cc, const uint32_t *h_ch, const hra_thresholds *th,
                    hra_part_result *results);

}  // namespace hra
