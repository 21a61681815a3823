// tb_sim.hip -- the particle updates of a leapfrog step around the tree build.
//
// The paper evaluates the construction inside N-body runs: a leapfrog
// integrator over constant timesteps, the tree rebuilt every step (Sec. 3),
// and notes that reordering the particles in memory is optional and may be
// done only every few steps (Sec. 2.3, Sec. 4).  Two kernels serve such a run:
//
// k_kick_drift : v += a dt_kick, then x += v dt_drift, for the particle at each
//                sorted position (the accelerations come out of the walk in key
//                order; perm maps them back to the caller's particle order);
// k_permute    : gathers rows of 4-byte words by perm, which reorders the
//                caller's particle arrays into key order.
//
// Both are plain streams over the particles (the kick's accesses through perm
// are sequential when the arrays were reordered recently, random otherwise).
#include "tb_internal.h"

namespace tb {

constexpr int kSimThreads = 256;

__global__ __launch_bounds__(kSimThreads) void k_kick_drift(
    const int32_t *__restrict__ perm, const double *__restrict__ acc, int64_t n, double dt_kick,
    double dt_drift, float *__restrict__ pos, float *__restrict__ vel,
    int32_t *__restrict__ status_word) {
  bool bad = false;
  for (int64_t s = blockIdx.x * (int64_t)kSimThreads + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * kSimThreads) {
    const int64_t i = perm ? (int64_t)perm[s] : s;
    if (i < 0 || i >= n) {
      bad = true;
      continue;
    }
    const double4 a = reinterpret_cast<const double4 *>(acc)[s];
    const double av[3] = {a.x, a.y, a.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      // FP64 update, one rounding per operation, stored in FP32
      const float v = (float)__dadd_rn((double)vel[3 * i + k], __dmul_rn(av[k], dt_kick));
      vel[3 * i + k] = v;
      pos[3 * i + k] = (float)__dadd_rn((double)pos[3 * i + k], __dmul_rn((double)v, dt_drift));
    }
  }
  if (status_word && __ballot(bad) != 0 && lane_id() == 0)
    atomicOr(status_word, TB_STATUS_INTERNAL);
}

__global__ __launch_bounds__(kSimThreads) void k_permute(const int32_t *__restrict__ perm,
                                                        int64_t n, const uint32_t *__restrict__ src,
                                                        int32_t width, uint32_t *__restrict__ dst,
                                                        int32_t *__restrict__ status_word) {
  bool bad = false;
  const int64_t total = n * width;
  for (int64_t e = blockIdx.x * (int64_t)kSimThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kSimThreads) {
    const int64_t s = e / width, k = e - s * width;
    const int64_t i = perm[s];
    if (i < 0 || i >= n) {
      bad = true;
      continue;
    }
    dst[e] = src[i * width + k];
  }
  if (status_word && __ballot(bad) != 0 && lane_id() == 0)
    atomicOr(status_word, TB_STATUS_INTERNAL);
}

static unsigned sim_grid(int64_t items) {
  int64_t g = (items + kSimThreads - 1) / kSimThreads;
  if (g > 8192) g = 8192;
  return (unsigned)(g < 1 ? 1 : g);
}

hipError_t launch_kick_drift(const int32_t *perm, const double *acc, int64_t n, double dt_kick,
                             double dt_drift, float *pos, float *vel, int32_t *status,
                             hipStream_t s) {
  k_kick_drift<<<sim_grid(n), kSimThreads, 0, s>>>(perm, acc, n, dt_kick, dt_drift, pos, vel,
                                                   status);
  return hipGetLastError();
}

hipError_t launch_permute(const int32_t *perm, int64_t n, const void *src, int32_t width,
                          void *dst, int32_t *status, hipStream_t s) {
  k_permute<<<sim_grid(n * width), kSimThreads, 0, s>>>(
      perm, n, static_cast<const uint32_t *>(src), width, static_cast<uint32_t *>(dst), status);
  return hipGetLastError();
}

}  // namespace tb
