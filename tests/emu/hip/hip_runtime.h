// Host stand-in for the HIP runtime header, used only by the host emulation
// test of the fused small-front kernels: a kernel launch runs its workgroups
// one after another, each as one std::thread per device thread, with
// __syncthreads() as a std::barrier, __shared__ variables as statics (one
// workgroup runs at a time) and the device atomics as host atomics.
#pragma once
#include <algorithm>
#include <atomic>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <thread>
#include <vector>

struct double2 {
  double x, y;
};
struct float2 {
  float x, y;
};
inline double2 make_double2(double a, double b) { return double2{a, b}; }
inline float2 make_float2(float a, float b) { return float2{a, b}; }

typedef int hipError_t;
typedef void* hipStream_t;
constexpr int hipSuccess = 0;
constexpr int hipErrorInvalidValue = 1;
inline hipError_t hipGetLastError() { return hipSuccess; }

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct EmuThreadIdx {
  static thread_local unsigned x;
};
inline thread_local unsigned EmuThreadIdx::x = 0;
struct EmuBlockIdx {
  static thread_local unsigned x;
};
inline thread_local unsigned EmuBlockIdx::x = 0;
#define threadIdx EmuThreadIdx()
#define blockIdx EmuBlockIdx()

inline std::barrier<>*& emu_barrier() {
  static std::barrier<>* b = nullptr;
  return b;
}
inline void __syncthreads() { emu_barrier()->arrive_and_wait(); }

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static

inline int atomicAdd(int* p, int v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
using std::fabs;
using std::fma;
using std::fmax;
using std::isfinite;
using std::max;
using std::min;

template <class K, class... A>
void emu_launch(K kernel, dim3 grid, dim3 block, A... args) {
  for (unsigned bx = 0; bx < grid.x; ++bx) {
    std::barrier<> bar(block.x);
    emu_barrier() = &bar;
    std::vector<std::thread> threads;
    for (unsigned t = 0; t < block.x; ++t)
      threads.emplace_back([&, t] {
        EmuThreadIdx::x = t;
        EmuBlockIdx::x = bx;
        kernel(args...);
      });
    for (auto& th : threads) th.join();
  }
}
#define hipLaunchKernelGGL(kernel, grid, block, shm, stream, ...) emu_launch(kernel, grid, block, __VA_ARGS__)
