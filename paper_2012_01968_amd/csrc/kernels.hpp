// Launch interface of the NTT kernels (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nttk {

struct Tw;
struct PassArgs;
struct VecDesc;

// Whether a (log2 N, log2 N1, OT stages) combination has kernels built in.
bool shape_supported(uint32_t logN, uint32_t logN1, int ot_stages);

// Whether a tile shape of the split passes has kernels built in and fits the split: row pass
// log2 values per lane (0 = default, 2, 3) and workgroup lanes (0 = default, 64, 128, 256);
// column pass width (0 = automatic, 16, 32, 64, 128 or 256 adjacent columns, at most N2).
bool tiles_supported(uint32_t logN, uint32_t logN1, uint32_t row_lr, uint32_t row_nth, uint32_t col_w);

// Forward / inverse transform of every vector described by `a`, enqueued on `st`.
hipError_t launch_forward(const PassArgs& a, int ot_stages, hipStream_t st);
hipError_t launch_inverse(const PassArgs& a, int ot_stages, hipStream_t st);

// One kernel of a transform: pass 0 / 1 in execution order (see ntt_forward_pass).
hipError_t launch_forward_pass(const PassArgs& a, int ot_stages, int pass, hipStream_t st);
hipError_t launch_inverse_pass(const PassArgs& a, int ot_stages, int pass, hipStream_t st);

// Row passes of a product with an NTT-domain key (forward row stages, key product, inverse
// row stages in one launch); `af` holds the forward tables and the keys, `ai` the inverse
// tables.  With logN1 = 0 this is the whole product; otherwise the forward column pass
// comes before it and the inverse column pass after it.
hipError_t launch_mul_rows(const PassArgs& af, const PassArgs& ai, int ot_stages, hipStream_t st);

// Fused single-launch transform (both passes, XCD-local queues); see fused.hpp.
struct FusedArgs;
bool fused_supported(uint32_t logN, uint32_t logN1, int ot_stages);
hipError_t launch_fused(const PassArgs& a, int ot_stages, bool inverse, uint32_t* ctr, uint32_t n_polys,
                        uint32_t lag, uint32_t max_grid, hipStream_t st);

// Transforms that keep the data in global memory between launches (stages.hip): one launch
// per group of log2_radix consecutive stages (1 = radix-2, one launch per stage).  Group g
// counts in execution order (the inverse runs the forward groups backwards).
uint32_t stage_group_count(uint32_t logN, int log2_radix);
hipError_t launch_stage_group(const PassArgs& a, int log2_radix, bool inverse, uint32_t g, hipStream_t st);
hipError_t launch_stage_groups(const PassArgs& a, int log2_radix, bool inverse, hipStream_t st);

// 32-bit words (kernels32.hip): primes below 2^30, tables of {w, floor(w 2^32 / q)} pairs.
bool shape32_supported(uint32_t logN, uint32_t logN1);
hipError_t launch_transform32(uint32_t* data, const void* tw, const void* scale, const uint32_t* q, uint64_t n_vec,
                              uint32_t L, uint32_t logN, uint32_t logN1, bool inverse, hipStream_t st);
hipError_t launch_pointwise32(const uint32_t* A, const uint32_t* B, uint32_t* C, const uint32_t* qs,
                              const uint64_t* mus, uint64_t n, uint32_t logN, uint32_t L, hipStream_t st);

// RNS <-> integer conversion (crt.hip): integers as [n_polys][W][N] little-endian words.
hipError_t launch_rns_decompose(const uint64_t* words, uint32_t W, uint64_t* res, uint32_t n_polys, uint32_t logN,
                                uint32_t L, const Tw* pow2, uint32_t pow2_stride, const uint64_t* qs, hipStream_t st);
hipError_t launch_crt_reconstruct(const uint64_t* res, uint64_t* out, uint32_t n_polys, uint32_t logN, uint32_t L,
                                  uint32_t W, const Tw* inv, const uint64_t* M, const uint64_t* kQ, const uint64_t* qs,
                                  hipStream_t st);

// In-place bit-reversal permutation of every vector described by `a` (slot i <-> slot
// brv(i)): turns the forward transform's bit-reversed output into natural order and back.
hipError_t launch_brv_permute(const PassArgs& a, hipStream_t st);

// Every vector of a list times its key vector, in place (Barrett products).
hipError_t launch_pointwise_list(const VecDesc* vecs, uint64_t n_vec, uint32_t logN, const uint64_t* qs,
                                 const uint64_t* mus, const uint32_t* bits, hipStream_t st);

// C = A * B mod q_l element-wise over n_elems elements of a [n_vec][N] batch.
hipError_t launch_pointwise(const uint64_t* A, const uint64_t* B, uint64_t* C, const uint64_t* qs,
                            const uint64_t* mus, const uint32_t* bits, uint64_t n_elems, uint32_t logN,
                            uint32_t L, hipStream_t st);

}  // namespace nttk
