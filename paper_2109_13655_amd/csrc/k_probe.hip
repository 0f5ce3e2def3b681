// Measurement probe: the rate at which the GPU gathers random 512-byte rows
// of a table and sums them, the access pattern of the sparse products of the
// block step (each output row of U = A Q or W = A^T U adds the gathered rows
// of its nonzeros) without the matrix values and indices.  It gives the
// ceiling a sparse product of that shape can reach on this memory system.
#include <random>
#include <vector>

#include "../../include/csvd_diag.h"
#include "csvd_impl.h"

namespace csvd {
namespace {

typedef double v2d __attribute__((ext_vector_type(2)));
constexpr int kRowD = 64;  // doubles per table row (512 bytes)

// variant 0: the lane layout of the block products (16 lanes per output row,
// lane c holds columns 4c..4c+3, two 16-byte loads per gathered row)
__global__ __launch_bounds__(kThreads) void k_gather_lane4(const double *__restrict__ tab,
                                                           const int *__restrict__ idx, int per_out,
                                                           int64_t out_rows, double *__restrict__ out) {
  constexpr int LPR = kRowD / 4, RPT = kThreads / LPR, UNR = 4;
  for (int64_t tile = blockIdx.x; tile * RPT < out_rows; tile += gridDim.x) {
    const int t = threadIdx.x, c0 = (t % LPR) * 4;
    const int64_t row = tile * RPT + t / LPR;
    if (row >= out_rows) continue;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int *ir = idx + row * per_out;
    int p = 0;
    for (; p + UNR <= per_out; p += UNR) {
      v2d xv[UNR][2];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const v2d *xp = reinterpret_cast<const v2d *>(tab + (int64_t)ir[p + u] * kRowD + c0);
        xv[u][0] = xp[0];
        xv[u][1] = xp[1];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        acc[0] += xv[u][0].x;
        acc[1] += xv[u][0].y;
        acc[2] += xv[u][1].x;
        acc[3] += xv[u][1].y;
      }
    }
    for (; p < per_out; ++p) {
      const v2d *xp = reinterpret_cast<const v2d *>(tab + (int64_t)ir[p] * kRowD + c0);
      const v2d x0 = xp[0], x1 = xp[1];
      acc[0] += x0.x;
      acc[1] += x0.y;
      acc[2] += x1.x;
      acc[3] += x1.y;
    }
    v2d *yp = reinterpret_cast<v2d *>(out + row * kRowD + c0);
    yp[0] = v2d{acc[0], acc[1]};
    yp[1] = v2d{acc[2], acc[3]};
  }
}

// variant 1: each load instruction of a row covers one contiguous half row
// (lane c reads columns 2c, 2c+1 and 32+2c, 32+2c+1)
__global__ __launch_bounds__(kThreads) void k_gather_half(const double *__restrict__ tab,
                                                          const int *__restrict__ idx, int per_out,
                                                          int64_t out_rows, double *__restrict__ out) {
  constexpr int LPR = kRowD / 4, RPT = kThreads / LPR, UNR = 4;
  for (int64_t tile = blockIdx.x; tile * RPT < out_rows; tile += gridDim.x) {
    const int t = threadIdx.x, c0 = (t % LPR) * 2;
    const int64_t row = tile * RPT + t / LPR;
    if (row >= out_rows) continue;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int *ir = idx + row * per_out;
    int p = 0;
    for (; p + UNR <= per_out; p += UNR) {
      v2d xv[UNR][2];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const double *b = tab + (int64_t)ir[p + u] * kRowD;
        xv[u][0] = *reinterpret_cast<const v2d *>(b + c0);
        xv[u][1] = *reinterpret_cast<const v2d *>(b + 32 + c0);
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        acc[0] += xv[u][0].x;
        acc[1] += xv[u][0].y;
        acc[2] += xv[u][1].x;
        acc[3] += xv[u][1].y;
      }
    }
    for (; p < per_out; ++p) {
      const double *b = tab + (int64_t)ir[p] * kRowD;
      const v2d x0 = *reinterpret_cast<const v2d *>(b + c0), x1 = *reinterpret_cast<const v2d *>(b + 32 + c0);
      acc[0] += x0.x;
      acc[1] += x0.y;
      acc[2] += x1.x;
      acc[3] += x1.y;
    }
    *reinterpret_cast<v2d *>(out + row * kRowD + c0) = v2d{acc[0], acc[1]};
    *reinterpret_cast<v2d *>(out + row * kRowD + 32 + c0) = v2d{acc[2], acc[3]};
  }
}

__global__ void k_fill_table(double *tab, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    tab[i] = (double)(i % 1021) * 0.5;
}

}  // namespace
}  // namespace csvd

using namespace csvd;

extern "C" int csvd_probe_gather(int64_t table_rows, int32_t variant, int64_t out_rows, int32_t per_out,
                                 uint64_t seed, int32_t reps, double *ms_per_launch) {
  if (table_rows < 1 || out_rows < 1 || per_out < 1 || reps < 1 || !ms_per_launch || variant < 0 || variant > 1)
    return CSVD_EINVAL;
  if (table_rows >= ((int64_t)1 << 31) || out_rows * per_out >= ((int64_t)1 << 34)) return CSVD_EINVAL;
  // random row indices, drawn on the host (each output row's list sorted,
  // like the column indices of a CSR row)
  std::vector<int> idx((size_t)(out_rows * per_out));
  std::mt19937_64 g(seed);
  std::uniform_int_distribution<int64_t> d(0, table_rows - 1);
  for (int64_t r = 0; r < out_rows; ++r) {
    int *ir = idx.data() + r * per_out;
    for (int p = 0; p < per_out; ++p) ir[p] = (int)d(g);
    std::sort(ir, ir + per_out);
  }
  double *tab = nullptr, *out = nullptr;
  int *didx = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = CSVD_OK;
  float ms = 0.f;
  const int64_t tiles = (out_rows + 15) / 16;
  const int grid = (int)std::min<int64_t>(tiles, 16384);
  auto launch = [&]() {
    if (variant == 0)
      hipLaunchKernelGGL(k_gather_lane4, dim3(grid), dim3(kThreads), 0, nullptr, tab, didx, per_out, out_rows, out);
    else
      hipLaunchKernelGGL(k_gather_half, dim3(grid), dim3(kThreads), 0, nullptr, tab, didx, per_out, out_rows, out);
  };
  if (hipMalloc(&tab, sizeof(double) * table_rows * kRowD) != hipSuccess ||
      hipMalloc(&out, sizeof(double) * out_rows * kRowD) != hipSuccess ||
      hipMalloc(&didx, sizeof(int) * idx.size()) != hipSuccess) {
    rc = CSVD_ENOMEM;
    goto done;
  }
  if (hipMemcpy(didx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = CSVD_EDEVICE;
    goto done;
  }
  hipLaunchKernelGGL(k_fill_table, dim3(4096), dim3(kThreads), 0, nullptr, tab, table_rows * kRowD);
  launch();
  launch();
  (void)hipEventRecord(e0, nullptr);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, nullptr);
  if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
      hipGetLastError() != hipSuccess) {
    rc = CSVD_EDEVICE;
    goto done;
  }
  *ms_per_launch = ms / reps;
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (tab) (void)hipFree(tab);
  if (out) (void)hipFree(out);
  if (didx) (void)hipFree(didx);
  return rc;
}
