// rmc_launch.h -- host-callable launchers of the kernels in rmc_kernels.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rmc_device.h"

namespace rmc {

// defer: peel-off rays past their first leaf go to the queue of
// d_probs[0].pq (then launch_peel_drain must follow).  one_line: every
// problem of the launch has a single line (a kernel specialised for it).
// regroup (with defer): one rejection round of a line scattering per pass
// of the loop, a rejected round leaving the event pending for the next.
// tail (single problem, defer): the kernel compiled for one wave per SIMD,
// for grids of at most one wave per SIMD.
hipError_t launch_transport(bool fp32, bool batch, bool defer, bool one_line, bool regroup, const ProblemK *d_probs,
                            const int64_t *d_starts, int n_probs, unsigned long long *d_next, int refill_min,
                            int stack_levels, int grid, int block, void *slots, int budget,
                            unsigned long long *slice, hipStream_t st, bool tail = false);
size_t slot_bytes();
// Ray-cast pass over the peel-off queue pq (a device PeelQueue), then the
// queue reset; grid blocks of 256 threads.
hipError_t launch_peel_drain(bool fp32, bool batch, bool one_line, const ProblemK *d_probs, void *pq,
                             int stack_levels, int grid, unsigned long long *slice, hipStream_t st);
int peel_drain_blocks_per_cu(bool fp32, bool batch, bool one_line, int stack_levels);
size_t peel_job_bytes(bool fp32);
size_t peel_queue_bytes();
int transport_blocks_per_cu(bool fp32, bool batch, bool defer, bool one_line, bool regroup, int block,
                            int stack_levels);
hipError_t launch_clear_slots(void *slots, int64_t n, hipStream_t st);
hipError_t launch_count_live(const void *slots, int64_t n, unsigned long long *out, hipStream_t st);
// active slots of src[0, n) copied to distinct slots of dst; *n_live += their count
hipError_t launch_compact_slots(const void *src, int64_t n, void *dst, unsigned long long *n_live,
                                hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);
hipError_t launch_trace(const ProblemK &pb, int64_t n, const double *orig, const double *dir,
                        int max_cells, int32_t *leaf, double *seg, int32_t *cnt, hipStream_t st);
hipError_t launch_tau(bool fp32, const ProblemK &pb, int64_t n, const double *orig, const double *dir,
                      const double *x, double *tau, hipStream_t st);
hipError_t launch_image_fwd(bool fp32, const ProblemK &pb, int obs, int64_t n, const double *orig,
                            const double *x, const double *w, double *image, unsigned long long *ncross,
                            hipStream_t st);
hipError_t launch_image_bwd(bool fp32, const ProblemK &pb, int obs, int64_t n, const double *orig,
                            const double *x, const double *w, const double *G, double inv_vth_ref,
                            double *gn, double *gk, double *gv, unsigned long long *ncross, hipStream_t st);
// Tape-recording image pass and its adjoint (the tape's per-wave arrays
// hold tape_waves(n) entries: every wave of the launch grid).
int64_t tape_waves(int64_t n);
hipError_t launch_image_fwd_tape(bool fp32, const ProblemK &pb, int obs, int64_t n, const double *orig,
                                 const double *x, const double *w, double *image, unsigned long long *ncross,
                                 const TapeK &tp, hipStream_t st);
hipError_t launch_image_bwd_tape(bool fp32, const ProblemK &pb, int obs, int64_t n, const TapeK &tp,
                                 const double *G, double inv_vth_ref, double *gn, double *gk, double *gv,
                                 unsigned long long *ncross, hipStream_t st);
// Gas given as float (f32_in) or double arrays on the device, checked and
// copied into raw[8n] (bad[0]: first invalid leaf, bad[1]: first leaf with
// |v_d| >= 0.1 c; both must start at ~0).
hipError_t launch_stage_gas(bool f32_in, int64_t n, const void *nh, const void *tk, const void *v, const void *kd,
                           double *raw, unsigned long long *bad, hipStream_t st);
// Leaf records (float when fp32) from raw gas and the leaves' levels and
// integer coordinates.
hipError_t launch_leaf_records(bool fp32, int64_t n, const double *raw, const int8_t *lv, const int32_t *ijk,
                               double T_ref, double vth_ref, double box, int domain, const double dom[4],
                               void *leaves, hipStream_t st);
// bad[0]: first source outside the box, with non-finite x or a non-unit
// direction (dir may be null); must start at ~0.
hipError_t launch_check_sources(int64_t n, const double *pos, const double *dir, const double *x,
                                unsigned long long *bad, hipStream_t st);
// g_v[3n] = g_vlos[n] k (velocity-vector gradient from the line-of-sight one)
hipError_t launch_vlos_to_v(int64_t n, const double *g_vlos, const double k[3], double *g_v, hipStream_t st);
// Counters the allocation-free spectrum call uses: the current device's
// copy of a fixed array of NOALLOC_MAX_BINS unsigned 64-bit counters
// (hipGetSymbolAddress, once per device; call with that device current).
constexpr int NOALLOC_MAX_BINS = 1 << 16;
hipError_t scratch_address(int device, unsigned long long **out);
hipError_t launch_hist(int64_t n, const int32_t *status, const double *x, int nbins, double x_min, double span,
                       unsigned long long *h, hipStream_t st);
hipError_t launch_batch_reset(const ProblemK *d_probs, int n, unsigned long long *d_next, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t st);
hipError_t launch_u64_to_f64(const unsigned long long *a, double *b, int64_t n, hipStream_t st);
hipError_t launch_f32_to_f64(const float *a, double *b, int64_t n, hipStream_t st);
hipError_t launch_f64_to_f32(const double *a, float *b, int64_t n, hipStream_t st);
// emitted x of packets [first, first+n) under the problem's source spectrum
hipError_t launch_source_x(bool f32, const ProblemK &pb, const double *src_x, double *x_out, int64_t first,
                           int64_t n, hipStream_t stream);

}  // namespace rmc
