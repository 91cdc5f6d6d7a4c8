// Pieces shared by the strip kernels (forward step and adjoint step): the
// strip geometry, buffer-resource constants, compile-time loops, the lane
// exchange and the XCD-aware workgroup order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace pclb {
namespace strip {

constexpr int WAVE = 64;                       // one strip = 64 theta columns, one per lane
// word 3 of a raw buffer resource on gfx9-family GPUs (32-bit data format)
constexpr int BUF_DWORD3 = 0x00020000;
constexpr int NXCD = 8;   // accelerator dies; workgroups are dealt to them round-robin
// Byte offset beyond the buffers' range: a raw buffer access at this offset
// is discarded by the hardware range check (a load returns 0).  Used for the
// stores of lanes past the last column, the look-ahead loads past a chunk's
// last row and the halo loads of lanes that read no halo, so that none of them
// needs a branch.
constexpr uint32_t OOB = 0x80000000u;
// Cache policy of the output stores: nontemporal (bit 1 on gfx950).  The new
// state is not read again in this launch, so it should not displace the input
// lines that the neighbouring strips still read as their azimuthal halo.
constexpr int STORE_NT = 2;

template <int V, int N, class Fn>
__device__ inline void for_v(Fn&& fn) {
  if constexpr (V < N) {
    fn(std::integral_constant<int, V>{});
    for_v<V + 1, N>(fn);
  }
}

__device__ inline float lane_from(float v, int byte_addr) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(byte_addr, __float_as_int(v)));
}

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7fffffff, BUF_DWORD3);
}

// Work item of this workgroup.  Workgroups are dealt to the XCDs
// round-robin; with xcd_order the ones that land on one XCD take a contiguous
// range of work items (work items run over strips first, then chunks), so that
// strips next to each other in theta, which read the same cache lines at their
// common edge, share that XCD's L2.
__device__ inline int work_item(int xcd_order) {
  int w = blockIdx.x;
  if (xcd_order) {
    const int nb = gridDim.x, per = nb / NXCD, extra = nb % NXCD;
    const int x = blockIdx.x % NXCD, local = blockIdx.x / NXCD;
    w = x * per + min(x, extra) + local;
  }
  return w;
}

inline int n_strips(int nth) { return (nth + WAVE - 1) / WAVE; }

}  // namespace strip
}  // namespace pclb
