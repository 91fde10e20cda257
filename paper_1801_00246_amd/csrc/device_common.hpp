// Device-side helpers shared by the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ipdg {

// Connectivity record of one element.  nb[f]: element across face f (the
// element itself on a boundary face).  info: bits 2f..2f+1 hold the
// neighbour's local index of the shared face, bits 8+2f..9+2f the boundary
// flag of face f (0 interior, 1 Dirichlet, 2 Neumann).
struct alignas(16) Conn {
  int nb[3];
  int info;
};

__host__ __device__ inline int conn_fp(int info, int f) { return (info >> (2 * f)) & 3; }
__host__ __device__ inline int conn_bc(int info, int f) { return (info >> (8 + 2 * f)) & 3; }

// Block of a batched launch (one launch running the same kernel for many
// solves): member s, its member-local block b of nb (the grid of the
// member's own launch) and, for element kernels, the tile stride of that
// grid's die mapping.
struct BlockRef {
  int s, b, nb, per;
};

constexpr int kBlock = 256;   // threads per block of the element kernels
constexpr int kXcd = 8;       // accelerator complex dies of an MI355X

// Block b of a launch of kXcd * per blocks -> tile index.  Blocks are
// dispatched round-robin over the dies, so consecutive tiles (which share
// neighbour data) are given to blocks that land on the same die and L2.
__device__ __forceinline__ int xcd_tile(int b, int per) { return (b % kXcd) * per + b / kXcd; }

inline int xcd_grid(int ntiles, int& per) {
  per = (ntiles + kXcd - 1) / kXcd;
  return per * kXcd;
}

#ifdef __HIPCC__
// A pointer read from an argument table in device memory (a batched launch)
// carries no address space, so loads through it would be generic (flat) and
// never scalar.  These casts restore what a kernel argument gets: global
// memory, or constant memory for read-only tables (wave-uniform loads from it
// become scalar loads).
// (Through an integer: a direct cast pair folds back to the generic pointer.)
template <typename T>
__device__ __forceinline__ T* in_global(T* p) {
  return (T*)((__attribute__((address_space(1))) T*)(unsigned long long)p);
}
template <typename T>
__device__ __forceinline__ const T* in_constant(const T* p) {
  return (const T*)((const __attribute__((address_space(4))) T*)(unsigned long long)p);
}

// outward face vector of face f: its direction is the unit normal and its
// length the face scale |F| / |E|
__device__ __forceinline__ void face_vec(int f, double rx, double sx, double ry, double sy, double& ax, double& ay) {
  if (f == 0) {
    ax = -sx;
    ay = -sy;
  } else if (f == 1) {
    ax = rx + sx;
    ay = ry + sy;
  } else {
    ax = -rx;
    ay = -ry;
  }
}

// Sum of v over the block, valid in thread 0.  Fixed reduction order, so the
// result is bitwise reproducible for a given launch shape.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
  __shared__ double red[kBlock / 64][NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    v[k] = s;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = red[0][k];
#pragma unroll
      for (int ww = 1; ww < kBlock / 64; ++ww) s += red[ww][k];
      v[k] = s;
    }
  }
}
#endif  // __HIPCC__

}  // namespace ipdg
