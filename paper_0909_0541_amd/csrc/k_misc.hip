// FP64 direct-summation judge (Eq. 1), leapfrog kick/drift and energy sums.
#include <mutex>

#include "bh_device.h"

namespace bh {

namespace {

constexpr int kJudgeI = 64;      // sampled particles per block (one per lane)
constexpr int kJudgeTile = 256;  // j particles staged in LDS per step

// Block (ib, jb): sampled particles ib*64 .. +63 against the j chunk jb.
// Partial sums are written per chunk and reduced in chunk order, so the
// result does not depend on scheduling.
__global__ __launch_bounds__(kJudgeI) void k_direct_partial(const double *__restrict__ pos, const double *__restrict__ mass,
                                                            int64_t n, double eps2, int64_t s,
                                                            const int64_t *__restrict__ idx, int64_t chunk,
                                                            double *__restrict__ part) {
  __shared__ double tj[kJudgeTile][4];
  const int64_t k = (int64_t)blockIdx.x * kJudgeI + threadIdx.x;
  const int64_t jb = blockIdx.y;
  const int64_t j0 = jb * chunk, j1 = min(n, j0 + chunk);
  int64_t i = -1;
  double xi = 0.0, yi = 0.0, zi = 0.0;
  if (k < s) {
    i = idx[k];
    xi = pos[3 * i];
    yi = pos[3 * i + 1];
    zi = pos[3 * i + 2];
  }
  double ax = 0.0, ay = 0.0, az = 0.0, p = 0.0;
  for (int64_t jt = j0; jt < j1; jt += kJudgeTile) {
    __syncthreads();
    for (int t = threadIdx.x; t < kJudgeTile; t += kJudgeI) {
      int64_t j = jt + t;
      if (j < j1) {
        tj[t][0] = pos[3 * j];
        tj[t][1] = pos[3 * j + 1];
        tj[t][2] = pos[3 * j + 2];
        tj[t][3] = mass[j];
      }
    }
    __syncthreads();
    const int nt = (int)min((int64_t)kJudgeTile, j1 - jt);
    for (int t = 0; t < nt; ++t) {
      if (jt + t == i) continue;
      const double dx = tj[t][0] - xi, dy = tj[t][1] - yi, dz = tj[t][2] - zi;
      const double r2 = dx * dx + dy * dy + dz * dz + eps2;
      const double rinv = 1.0 / sqrt(r2);
      const double mr = tj[t][3] * rinv;
      const double mr3 = mr * rinv * rinv;
      ax += mr3 * dx;
      ay += mr3 * dy;
      az += mr3 * dz;
      p += mr;
    }
  }
  if (k < s) {
    double *q = part + 4 * (jb * s + k);
    q[0] = ax;
    q[1] = ay;
    q[2] = az;
    q[3] = p;
  }
}

__global__ void k_direct_reduce(const double *__restrict__ part, int64_t s, int64_t nchunk, double *__restrict__ acc,
                                double *__restrict__ pot) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= s) return;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t c = 0; c < nchunk; ++c)
    for (int q = 0; q < 4; ++q) a[q] += part[4 * (c * s + k) + q];
  acc[3 * k] = a[0];
  acc[3 * k + 1] = a[1];
  acc[3 * k + 2] = a[2];
  pot[k] = -a[3];
}

__global__ void k_kick(int64_t n, double *__restrict__ vel, const float *__restrict__ acc, double dt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n) return;
  vel[i] += dt * (double)acc[i];
}

__global__ void k_drift(int64_t n, double *__restrict__ pos, const double *__restrict__ vel, double dt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n) return;
  pos[i] += dt * vel[i];
}

constexpr int kEnergyBlocks = 1024;

__global__ __launch_bounds__(256) void k_energy_partial(int64_t n, const double *__restrict__ vel,
                                                        const double *__restrict__ mass, const float *__restrict__ pot,
                                                        double *__restrict__ part) {
  __shared__ double red[2][256];
  double ek = 0.0, ep = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
    ek += 0.5 * mass[i] * (vx * vx + vy * vy + vz * vz);
    ep += 0.5 * mass[i] * (double)pot[i];
  }
  red[0][threadIdx.x] = ek;
  red[1][threadIdx.x] = ep;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}

__global__ void k_energy_final(const double *__restrict__ part, int nb, double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < nb; ++k) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  out[0] = a;
  out[1] = b;
}

}  // namespace

// The judge's partial sums for callers that cannot allocate
// (bh_direct_sampled_noalloc): one static array per device, held until the
// process ends.  Host code never names it except to look up its device
// address (judge_scratch_address); every call on a device shares it.
static __device__ __align__(256) double scratch[kJudgeScratchBytes / sizeof(double)];

hipError_t judge_scratch_address(int device, double **ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double *addr[kMaxDevices] = {};
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = static_cast<double *>(p);
  }
  *ptr = addr[device];
  return hipSuccess;
}

size_t direct_part_bytes(int64_t n, int64_t s, int num_cu, int64_t *chunk, int64_t *nchunk) {
  // enough j chunks that the grid holds a few blocks per compute unit
  const int64_t iblocks = (s + kJudgeI - 1) / kJudgeI;
  int64_t want = (int64_t)num_cu * 8 / (iblocks > 0 ? iblocks : 1);
  if (want < 1) want = 1;
  int64_t c = (n + want - 1) / want;
  if (c < kJudgeTile) c = kJudgeTile;
  *chunk = c;
  *nchunk = (n + c - 1) / c;
  if (*nchunk < 1) *nchunk = 1;
  return (size_t)(*nchunk) * (size_t)s * 4 * sizeof(double);
}

void direct_sampled_device(const double *pos, const double *mass, int64_t n, double eps, int64_t s,
                           const int64_t *idx, double *acc, double *pot, double *part, int64_t chunk,
                           int64_t nchunk, hipStream_t st) {
  if (s <= 0) return;
  dim3 grid((unsigned)((s + kJudgeI - 1) / kJudgeI), (unsigned)nchunk);
  k_direct_partial<<<grid, kJudgeI, 0, st>>>(pos, mass, n, eps * eps, s, idx, chunk, part);
  k_direct_reduce<<<(unsigned)((s + 255) / 256), 256, 0, st>>>(part, s, nchunk, acc, pot);
}

void kick_device(int64_t n, double *vel, const float *acc, double dt, hipStream_t s) {
  if (n > 0) k_kick<<<(unsigned)((3 * n + 255) / 256), 256, 0, s>>>(n, vel, acc, dt);
}

void drift_device(int64_t n, double *pos, const double *vel, double dt, hipStream_t s) {
  if (n > 0) k_drift<<<(unsigned)((3 * n + 255) / 256), 256, 0, s>>>(n, pos, vel, dt);
}

size_t energy_part_bytes() { return (size_t)kEnergyBlocks * 2 * sizeof(double); }

void energy_device(int64_t n, const double *vel, const double *mass, const float *pot, double *part, double *out,
                   hipStream_t s) {
  k_energy_partial<<<kEnergyBlocks, 256, 0, s>>>(n, vel, mass, pot, part);
  k_energy_final<<<1, 64, 0, s>>>(part, kEnergyBlocks, out);
}

}  // namespace bh
