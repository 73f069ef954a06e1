// launch.h -- host-side launchers of the correlation kernels and the job
// sources they read (inline in the kernel arguments for a single call, or a
// device array for a batch).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "corr2d_internal.h"

namespace corr2d {

// Up to two jobs passed by value; blocks [0, blocks0) belong to job 0.
struct TableSrcInline {
    TableJob j[2];
    int32_t blocks0;
    int32_t count;
    int* counter;       // unused (nullptr); the batched source resets its ticket counters
    int32_t ncounters;  // 0
    __device__ TableJob get(int b, int& lb) const {
        if (count == 1 || b < blocks0) { lb = b; return j[0]; }
        lb = b - blocks0;
        return j[1];
    }
    // workgroup b of the Q N kernel (one job: the single and hetero plans
    // share one table)
    __device__ TableJob get_q(int b, int& lb) const { lb = b; return j[0]; }
};

// Jobs in device memory; start[q] is the first block of job q (count + 1
// entries, start[count] = total blocks).
struct TableSrcArray {
    const TableJob* jobs;
    const int32_t* start;
    const int32_t* qstart;  // first Q N workgroup of job q (count + 1 entries)
    int32_t count;
    int32_t ncounters;  // ticket counters of the persistent launches (one per tile shape)
    int* counter;       // set to 0 by block 0
    __device__ static int find(const int32_t* st, int count, int b) {
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (st[mid] <= b) lo = mid;
            else hi = mid - 1;
        }
        return lo;
    }
    __device__ TableJob get(int b, int& lb) const {
        const int q = find(start, count, b);
        lb = b - start[q];
        return jobs[q];
    }
    __device__ TableJob get_q(int b, int& lb) const {
        const int q = find(qstart, count, b);
        lb = b - qstart[q];
        return jobs[q];
    }
};

struct PrepSrcInline {
    PrepJob j[2];
    int32_t blocks0;
    int32_t count;
    __device__ PrepJob get(int b, int& lb) const {
        if (count == 1 || b < blocks0) { lb = b; return j[0]; }
        lb = b - blocks0;
        return j[1];
    }
};

struct PrepSrcArray {
    const PrepJob* jobs;
    const int32_t* start;
    int32_t count;
    int32_t pad;
    __device__ PrepJob get(int b, int& lb) const {
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (start[mid] <= b) lo = mid;
            else hi = mid - 1;
        }
        lb = b - start[lo];
        return jobs[lo];
    }
};

// max_m: the largest perturbation length among the jobs (sizes the LDS)
hipError_t launch_tables(const TableSrcInline& src, int blocks, int64_t max_m, hipStream_t s);
hipError_t launch_tables(const TableSrcArray& src, int blocks, int64_t max_m, hipStream_t s);
hipError_t launch_center(const PrepSrcInline& src, int blocks, hipStream_t s);
// tables (nt workgroups), their Q N rows (nq) and the centring (nc) in one
// launch, for m <= kPrepMergeMaxM (its dynamic LDS is 32 m bytes)
hipError_t launch_prep(const TableSrcInline& ts, int nt, int nq, int64_t m, const PrepSrcInline& ps, int nc,
                       hipStream_t s);
constexpr int64_t kPrepMergeMaxM = 1024;
hipError_t launch_center(const PrepSrcArray& src, int blocks, hipStream_t s);
hipError_t launch_transform(int prec, const PrepSrcInline& src, int blocks, hipStream_t s);
hipError_t launch_transform(int prec, const PrepSrcArray& src, int blocks, hipStream_t s);
// Centring fused into the FP32 transform GEMM (not FP64), for kt <=
// kFusedTransformMaxK; the same workgroups as launch_transform.
hipError_t launch_center_transform(int prec, const PrepSrcInline& src, int blocks, hipStream_t s);
hipError_t launch_center_transform(int prec, const PrepSrcArray& src, int blocks, hipStream_t s);
constexpr int kFusedTransformMaxK = 256;
// single calls fuse only with at least this many workgroups (two per CU)
constexpr int kFusedMinBlocks = 512;
// Radix FFT transform (power-of-two m, 128 <= m <= 1024, FFT length
// L = 2^log2l = 2m; fft_points(L) spectral points per workgroup: 8, or the
// 4096/L points of one pass of its 256 threads) and its tables (2m
// workgroups).
hipError_t launch_fft_tables(const TableSrcInline& src, int64_t m, hipStream_t s);
hipError_t launch_fft_transform(int prec, int log2l, const PrepSrcInline& src, int blocks, hipStream_t s);
constexpr int fft_points(int L) { return 4096 / L > 8 ? 4096 / L : 8; }
hipError_t launch_corr(int prec, int fm, int fn, const CorrJob& C, int64_t blocks, hipStream_t s);
hipError_t launch_corr_persistent(int prec, int fm, int fn, bool out_f64, const CorrJob* jobs,
                                  const int64_t* tile_start, int count, int64_t total,
                                  int* counter, int blocks, hipStream_t s);
int corr_variant_supported(int prec, int fm, int fn);
int persistent_blocks_per_cu(int prec, int fm, int fn, bool out_f64);
hipError_t launch_interp(const InterpJob& J, hipStream_t s);
hipError_t launch_row_select(const SelJob& J, hipStream_t s);
hipError_t launch_tables_qn(const TableSrcInline& src, int blocks, int64_t max_m, hipStream_t s);
hipError_t launch_tables_qn(const TableSrcArray& src, int blocks, int64_t max_m, hipStream_t s);
// Workgroups of the Q N kernel for one table: one per frequency 0..floor(m/2).
inline int qn_blocks(int64_t m) { return (int)(m / 2 + 1); }

}  // namespace corr2d
