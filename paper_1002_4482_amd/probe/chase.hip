// Measurement probe, not part of the solver library: the memory access
// pattern of the level-0 sublist walk without its work distribution and
// splitter tests, to give the walk a ceiling measured on the same chip.
//
// A lane follows a list from a start node for `hops` steps (or to the tail):
// x <- a[x], a dependent random 4-byte read per step.  With `write` set it
// also stores to the word it just read (a[x] = successor ^ salt; the caller
// passes salt 0, which the compiler cannot know), so every step reads and
// dirties one random line, as the walk does when it overwrites a successor
// with a node's packed state.  With starts[i] = the (i * hops)-th node of the
// list, the lanes' segments partition the list and every node is visited
// once.  Lanes are spread over a grid that fills the device, one segment at
// a time per lane.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

template <bool kWrite>
__global__ void __launch_bounds__(256) chase(int32_t* a, const int32_t* __restrict__ starts,
                                             int64_t r, int hops, int32_t salt,
                                             unsigned long long* visited) {
  unsigned long long count = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < r;
       i += (int64_t)gridDim.x * blockDim.x) {
    int x = starts[i];
    for (int h = 0; h < hops && x >= 0; ++h) {
      const int s = a[x];
      if (kWrite) a[x] = s ^ salt;
      ++count;
      x = s == x ? -1 : s;  // -1 or a self-loop ends the list
    }
  }
  for (int o = 32; o > 0; o >>= 1) count += __shfl_xor(count, o, 64);
  if ((threadIdx.x & 63) == 0 && count) atomicAdd(visited, count);
}

}  // namespace

extern "C" {

// Times one chase over r segments of `hops` steps on `stream` with HIP
// events: *ms receives the kernel's device time and *visited (host) the
// number of steps taken.  a: DEVICE int32[n] successor array (tail -1 or a
// self-loop), read and, with write != 0, rewritten to the same values;
// starts: DEVICE int32[r] node ids in range; scratch: DEVICE 8 bytes.
// Returns 0, or -1 on a bad argument / HIP error.
int pjp_chase(int32_t* a, const int32_t* starts, int64_t r, int32_t hops, int32_t write,
              int32_t salt, void* scratch, float* ms, unsigned long long* visited,
              hipStream_t stream) {
  if (!a || !starts || r <= 0 || hops <= 0 || !scratch || !ms || !visited) return -1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -1;
  int64_t g = (r + 255) / 256;
  const int64_t cap = (int64_t)cus * 8;  // 8 workgroups of 256 per CU: 2048 lanes per CU
  if (g > cap) g = cap;
  unsigned long long* d_vis = static_cast<unsigned long long*>(scratch);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1;
  int rc = 0;
  if (hipMemsetAsync(d_vis, 0, sizeof(unsigned long long), stream) != hipSuccess) rc = -1;
  if (rc == 0 && hipEventRecord(e0, stream) != hipSuccess) rc = -1;
  if (rc == 0) {
    if (write)
      hipLaunchKernelGGL(chase<true>, dim3((unsigned)g), dim3(256), 0, stream, a, starts, r, hops,
                         salt, d_vis);
    else
      hipLaunchKernelGGL(chase<false>, dim3((unsigned)g), dim3(256), 0, stream, a, starts, r,
                         hops, salt, d_vis);
    if (hipGetLastError() != hipSuccess) rc = -1;
  }
  if (rc == 0 && hipEventRecord(e1, stream) != hipSuccess) rc = -1;
  if (rc == 0 && hipEventSynchronize(e1) != hipSuccess) rc = -1;
  if (rc == 0 && hipEventElapsedTime(ms, e0, e1) != hipSuccess) rc = -1;
  if (rc == 0 &&
      hipMemcpy(visited, d_vis, sizeof(unsigned long long), hipMemcpyDeviceToHost) != hipSuccess)
    rc = -1;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // extern "C"
