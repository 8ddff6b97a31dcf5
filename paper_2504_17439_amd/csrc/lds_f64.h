// Direct-to-LDS staging of FP64 MFMA operands (v_mfma_f64_16x16x4_f64),
// shared by the GEMM engine and the fold of the self-energy stage.
//
// A wave instruction of buffer_load ... lds moves 16 bytes per lane (1 KB)
// into LDS at M0 + 16 * lane.  Lanes that must not read get a buffer offset
// past the resource's range and deposit zeros.
//
// Two LDS layouts (doubles), both free of bank conflicts for eight lanes of
// a b128 read and sixteen of a b64 read:
//   k-contiguous rows: row r at r * 16 (16 k per slab), its eight k pairs at
//     pair slot c ^ (r & 7); a fragment is one ds_read_b128 feeding two MFMAs;
//   k rows of W elements: element r of k row k at k * W + (r ^ sw(k)),
//     sw(k) = 16 ((k >> 1) & 3); a fragment is two ds_read_b64 (k, k + 1).
// Both order k the same way: MFMA e of k8-step h takes, in lane group
// g = lane >> 4, the k index 2 (4h + g) + e.
#pragma once

#include <hip/hip_runtime.h>

namespace gwm {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) void* lds_ptr_t;

constexpr unsigned LDS_MASKED = 0x7ffffff0u;   // buffer offset of a masked lane (>= the range: reads zero)
constexpr int LDS_NREC = 0x7ffffff0;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t f64_rsrc(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, LDS_NREC, 0x00020000);
}

// 16 bytes per lane: one wave instruction fills 1 KB of LDS at lds + 16 * lane
__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t rs, double* lds, unsigned voff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr_t)lds, 16, voff, 0, 0, 0);
}

__device__ __forceinline__ int ksw(int k) { return 16 * ((k >> 1) & 3); }

// Fragment of the k-contiguous rows rb .. rb + 15 for k8-step h.
__device__ __forceinline__ v2d frag_kc(const double* S, int rb, int h, int lane) {
    const int kp = 4 * h + (lane >> 4);
    const int r = rb + (lane & 15);
    return *(const v2d*)(S + r * 16 + ((kp ^ (r & 7)) << 1));
}

// Fragment of elements rb .. rb + 15 of k rows of W elements, k8-step h.
template <int W>
__device__ __forceinline__ v2d frag_kr(const double* S, int rb, int h, int lane) {
    const int k = 2 * (4 * h + (lane >> 4));
    const int rs = (rb + (lane & 15)) ^ ksw(k);
    v2d f;
    f.x = S[k * W + rs];
    f.y = S[(k + 1) * W + rs];
    return f;
}

}  // namespace gwm
