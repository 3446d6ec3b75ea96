// Host-side entry points into the kernels of fs_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fs_internal.hpp"

namespace fsk {

// Address of the fused step kernel for a storage/weights combination
// (launched with one StepArgs argument); mode is fsi::MODE_*: the LDS
// variants run RESIDENT_TPB threads, one workgroup per compute unit, the
// streaming variant STREAM_TPB threads per workgroup.
// udeg (StepArgs::udeg: a uniform layout's degree, or -1) selects the
// instantiation: mixed, or uniform with a preload depth of 8, 10 or 12;
// shed the one for age-dependent shedding (StepArgs::shed0/shed1/shed);
// extra the one that records rates (StepArgs::rates) and walks the
// active-chunk list of compaction (StepArgs::act, live).
// lgR: log2 of the replica count; sims with one replica (and neither
// shedding nor the extra checks) take an instantiation that knows it.
// pbits (StepArgs::pbits): packed columns (20, 24 or 27 bits; unit weights,
// one replica, not shedding together with the extra checks), or 0; nullptr
// for any other combination with pbits != 0.
const void* step_kernel_fn(int storage, bool weighted, int mode, int udeg, bool shed, bool extra, int lgR,
                           int pbits);
const void* step_kernel_fn_r1(int storage, bool weighted, int mode, int udeg);
const void* step_kernel_fn_r16(int storage, int mode, int udeg);
const void* step_kernel_fn_r1p20(int storage, int mode, int udeg);
const void* step_kernel_fn_r1p24(int storage, int mode, int udeg);
const void* step_kernel_fn_r1p27(int storage, int mode, int udeg);
const void* step_kernel_fn_shed_r1p20(int storage, int mode, int udeg);
const void* step_kernel_fn_shed_r1p24(int storage, int mode, int udeg);
const void* step_kernel_fn_shed_r1p27(int storage, int mode, int udeg);
const void* step_kernel_fn_extra_r1p20(int storage, int mode, int udeg);
const void* step_kernel_fn_extra_r1p24(int storage, int mode, int udeg);
const void* step_kernel_fn_extra_r1p27(int storage, int mode, int udeg);
// (the other (shed, extra) instantiations, each defined by a source of its own)
const void* step_kernel_fn_extra(int storage, bool weighted, int mode, int udeg);
const void* step_kernel_fn_shed(int storage, bool weighted, int mode, int udeg);
const void* step_kernel_fn_shed_extra(int storage, bool weighted, int mode, int udeg);
const void* heavy_kernel_fn_shed(bool weighted, bool resident);

// Exact counts of one replica: per-workgroup partials (at most max_grid rows
// of 4 in `part`) reduced into out4.
hipError_t launch_recount(int storage, const void* state, int32_t n, int32_t lgR, int32_t replica,
                          uint32_t* part, uint32_t max_grid, uint32_t* out4, hipStream_t s);
// Pushed pressure of the binned rows [hub_base, hub_base + hubs) from the
// bitmap `bits`: out[(row - hub_base) * R + r] = infectious in-neighbours of
// the row in replica r (StepArgs::hub_T).
hipError_t launch_hub_recount(const int32_t* row_ptr, const int32_t* col_ind, int32_t hub_base, uint32_t hubs,
                              int32_t lgR, const uint32_t* bits, uint32_t* out, hipStream_t s);
// reduce_kernel(Ctl*, const uint32_t* part, uint32_t G, uint32_t C, uint32_t* out, uint32_t H):
// one block per slot, RED_TPB threads; with a ctl it also adds the slot count (its
// grid) to the step index, which ends a launch sequence.
const void* reduce_kernel_fn();
// Segment partials of degree-binned rows (HeavyArgs): heavy_pressure_kernel
// (WG threads, bits from global memory), or with resident set
// heavy_resident_kernel (RESIDENT_TPB threads, at most one workgroup per CU,
// the bitmap copied into LDS).
const void* heavy_kernel_fn(bool weighted, bool shed, bool resident);
// summary_kernel(SumArgs): one thread per summary bit (sum_words * 64 threads
// in WG-thread workgroups).
const void* summary_kernel_fn();

// Batched launches over the members of an fs_batch (see the kernels for the
// block-to-member mapping):
// step_batch_kernel(const StepArgs* table, const uint32_t* first, uint32_t members, uint32_t step_off),
//   STREAM_TPB threads, first[members] workgroups;
const void* step_batch_kernel_fn(int storage, bool weighted, bool extra);
// heavy_batch_kernel(const HeavyArgs* table, const uint32_t* first, uint32_t members, uint32_t step_off), WG threads;
const void* heavy_batch_kernel_fn(bool weighted);
// reduce_batch_kernel(const RedArgs* table): grid (r, members), RED_TPB threads;
// advances every member's step index by r
const void* reduce_batch_kernel_fn();
hipError_t launch_put_replica(int storage, void* state, void* age, const int32_t* src_state, const void* src_age,
                              int32_t n, int32_t lgR, int32_t replica, hipStream_t s);
hipError_t launch_rebuild_bits(int storage, const void* state, uint32_t total, unsigned long long* bits,
                               uint32_t words, hipStream_t s);
hipError_t launch_get_replica(int storage, const void* state, const void* age, int32_t* dst_state,
                              void* dst_age, int32_t n, int32_t lgR, int32_t replica, hipStream_t s);
hipError_t launch_get_rates(const float* rates, float* dst, int32_t n, int32_t lgR, int32_t replica,
                            hipStream_t s);
hipError_t launch_seed(int storage, void* state, void* age, const int64_t* nodes, int64_t count, int32_t lgR,
                       int32_t replica, int32_t comp, hipStream_t s);
hipError_t launch_clear_u32(uint32_t* p, size_t n, hipStream_t s);
hipError_t launch_set_ctl(fsi::Ctl* ctl, unsigned long long step, hipStream_t s);
hipError_t launch_eval_hazard(const fsi::HazardDev& h, int32_t storage, const void* ages, float* out, int64_t n,
                              hipStream_t s);
// Hazards of both laws (hz: device memory, hz[0] and hz[1]) at the ages in
// tab[m].x into tab[m].y, .z (StepArgs::htab).
hipError_t launch_hazard_table(const fsi::HazardDev* hz, int32_t same_kind, float4* tab, uint32_t n, hipStream_t s);
hipError_t launch_eval_shed(const fsi::ShedDev& sd, int32_t storage, const void* ages, float* out, int64_t n,
                            hipStream_t s);
// s(tau) of the infectious units into out (others untouched).
hipError_t launch_rebuild_shed(int storage, const void* state, const void* age, uint32_t total,
                               const fsi::ShedDev& sd, void* out, hipStream_t s);
// Live flags of all nchunks chunks from the state.
hipError_t launch_chunk_live(int storage, const void* state, uint32_t total, uint8_t* live, uint32_t nchunks,
                             hipStream_t s);
// compact_refresh_kernel(const uint8_t* live, uint32_t nchunks, uint32_t rows, uint32_t n, uint32_t* act):
// one workgroup of WG_REFRESH threads; live padded with zeros to whole tiles of LIVE_TILE flags.
const void* compact_refresh_kernel_fn();
// clear_u32_kernel(uint32_t* p, size_t n): grid-stride zero fill, 256 threads.
const void* clear_u32_kernel_fn();
hipError_t launch_eval_philox(const uint4* ctr, uint32_t k0, uint32_t k1, uint4* out, int64_t n, hipStream_t s);

} // namespace fsk
