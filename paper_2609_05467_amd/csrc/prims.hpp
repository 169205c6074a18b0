// Device-wide primitives of the hierarchy build (bvh.hip) for the other
// stages: the stable LSD radix sort of (uint64 key, uint32 value) pairs
// (eight passes of eight bits; the result lands in k1/v1 when
// *result_in_k1, else in k0/v0) and the prefix sum over uint32, each with
// its workspace size in uint32 elements.  Both are stream-ordered and
// allocate nothing.
#pragma once

#include "common.hpp"

namespace hra {
int64_t sort_pairs_ws_elems(int64_t n);
// passes: the keys are ordered by their low 8 x passes bits.
hipError_t sort_pairs(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n, uint32_t *ws, hipStream_t s,
                      bool *result_in_k1, int passes = 8);
int64_t scan_u32_ws_elems(int64_t n);
// A spatial order of n samples: their indices sorted stably by a 21-bit
// Morton code of the origin in the part's box (7 bits per axis), written to
// order[n].  `ws` holds sample_order_ws_bytes(n) bytes.
size_t sample_order_ws_bytes(int64_t n);
hipError_t sample_order(const float *origin, int64_t n, const PartMeta *meta, int32_t *order, void *ws, hipStream_t s);
// The same over the samples of several parts (the one-sample hemisphere
// cast jobs of a batch, item = sample): keys are (job << 21) | the Morton
// code in the job's part box, so the order keeps parts apart.  k0/v0 and
// k1/v1 hold n keys and values each, ws sort_pairs_ws_elems(n) elements;
// *order receives whichever values array holds the result.
hipError_t sample_order_jobs(const CastJob *d_jobs, int32_t n_jobs, const CastJob &job0, int64_t n, uint64_t *k0,
                             uint32_t *v0, uint64_t *k1, uint32_t *v1, uint32_t *ws, hipStream_t s,
                             const int32_t **order);
hipError_t scan_u32(const uint32_t *in, uint32_t *out, int64_t n, bool inclusive, uint32_t *ws, hipStream_t s);
}  // namespace hra
