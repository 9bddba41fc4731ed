// ccake_bench -- native driver of the C ABI, with no Python or PyTorch in the
// process (for profilers that count hardware events per dispatch).
//
//   ccake_bench INPUT STEPS [WARMUP]
//       Loads a workload file written by `bench.py --write-inputs`, creates
//       the EoS table and one simulation in a hipMalloc'd workspace, runs
//       WARMUP steps, re-initialises, and times STEPS Heun steps on a
//       non-default stream.  Prints one JSON line.
//   ccake_bench --copy MIB
//       One device-to-device copy of MIB MiB by a plain copy kernel (read
//       MIB MiB, write MIB MiB): the reference dispatch for the HBM byte
//       counters.
//
// Workload file (little endian): "CCAKEBN1", the ccake_config struct as laid
// out in ccake.h, int64 n, double t0, double dt, int32 dens_kind, int32 pad,
// int32 table nodes[4], double lo[4], double hi[4], double cols[7][nodes],
// double xi[dim][n], double u[dim][n], double dens[4][n].
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ccake.h"

namespace {

#define CK(x)                                                                              \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) {                                                                \
      std::fprintf(stderr, "%s:%d %s: %s\n", __FILE__, __LINE__, #x, hipGetErrorString(e_)); \
      std::exit(2);                                                                        \
    }                                                                                      \
  } while (0)

#define CC(h, x)                                                                           \
  do {                                                                                     \
    ccake_status s_ = (x);                                                                 \
    if (s_ != CCAKE_OK) {                                                                  \
      std::fprintf(stderr, "%s failed (%d): %s\n", #x, s_, ccake_last_error(h));           \
      std::exit(3);                                                                        \
    }                                                                                      \
  } while (0)

__global__ void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

int copy_mode(long mib) {
  if (mib <= 0 || mib > (1L << 16)) {
    std::fprintf(stderr, "--copy: MIB must be in 1..65536\n");
    return 1;
  }
  const size_t bytes = (size_t)mib << 20;
  void *a = nullptr, *b = nullptr;
  CK(hipMalloc(&a, bytes));
  CK(hipMalloc(&b, bytes));
  CK(hipMemset(a, 1, bytes));
  CK(hipDeviceSynchronize());
  const int64_t n = (int64_t)(bytes / sizeof(uint4));
  hipLaunchKernelGGL(k_copy, dim3(4096), dim3(256), 0, 0, (const uint4*)a, (uint4*)b, n);
  CK(hipGetLastError());
  CK(hipDeviceSynchronize());
  std::printf("{\"copy_bytes\": %zu}\n", bytes);
  CK(hipFree(a));
  CK(hipFree(b));
  return 0;
}

template <class T>
void get(FILE* f, T* dst, size_t count, const char* what) {
  if (std::fread(dst, sizeof(T), count, f) != count) {
    std::fprintf(stderr, "truncated workload file (%s)\n", what);
    std::exit(1);
  }
}

}  // namespace

int main(int argc, char** argv) {
  if (argc >= 3 && std::strcmp(argv[1], "--copy") == 0) return copy_mode(std::atol(argv[2]));
  if (argc < 3) {
    std::fprintf(stderr, "usage: ccake_bench INPUT STEPS [WARMUP] | ccake_bench --copy MIB\n");
    return 1;
  }
  const int steps = std::atoi(argv[2]);
  const int warmup = argc > 3 ? std::atoi(argv[3]) : 10;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) {
    std::fprintf(stderr, "cannot open %s\n", argv[1]);
    return 1;
  }
  char magic[8];
  get(f, magic, 8, "magic");
  if (std::memcmp(magic, "CCAKEBN1", 8) != 0) {
    std::fprintf(stderr, "not a workload file\n");
    return 1;
  }
  ccake_config cfg;
  get(f, &cfg, 1, "config");
  int64_t n;
  double t0, dt;
  int32_t dens_kind, pad;
  get(f, &n, 1, "n");
  get(f, &t0, 1, "t0");
  get(f, &dt, 1, "dt");
  get(f, &dens_kind, 1, "dens_kind");
  get(f, &pad, 1, "pad");
  int32_t nodes[4];
  double lo[4], hi[4];
  get(f, nodes, 4, "nodes");
  get(f, lo, 4, "lo");
  get(f, hi, 4, "hi");
  const size_t nn = (size_t)nodes[0] * nodes[1] * nodes[2] * nodes[3];
  if (n <= 0 || n > (int64_t)1 << 31 || cfg.dim < 2 || cfg.dim > 3 || nn == 0 || nn > ((size_t)1 << 28)) {
    std::fprintf(stderr, "bad workload header\n");
    return 1;
  }
  std::vector<double> cols(7 * nn), xi((size_t)cfg.dim * n), u((size_t)cfg.dim * n), dens(4 * (size_t)n);
  get(f, cols.data(), cols.size(), "table");
  get(f, xi.data(), xi.size(), "xi");
  get(f, u.data(), u.size(), "u");
  get(f, dens.data(), dens.size(), "dens");
  std::fclose(f);

  ccake_eos* eos = nullptr;
  CC(nullptr, ccake_eos_create_table(&eos, nodes, lo, hi, cols.data(), 60, 1e-13));
  size_t bytes = 0;
  CC(eos, ccake_workspace_bytes(&cfg, n, &bytes));
  void* ws = nullptr;
  CK(hipMalloc(&ws, bytes));
  hipStream_t stream;
  CK(hipStreamCreate(&stream));
  ccake_sim* sim = nullptr;
  CC(eos, ccake_create(&sim, &cfg, eos, n, ws, bytes, stream));
  CC(sim, ccake_init_particles(sim, t0, xi.data(), u.data(), dens_kind, dens.data(), CCAKE_HOST));
  if (warmup > 0) {
    CC(sim, ccake_step(sim, dt, warmup));
    CC(sim, ccake_check(sim));
  }
  CC(sim, ccake_init_particles(sim, t0, xi.data(), u.data(), dens_kind, dens.data(), CCAKE_HOST));
  CK(hipStreamSynchronize(stream));
  const auto a = std::chrono::steady_clock::now();
  CC(sim, ccake_step(sim, dt, steps));
  CK(hipStreamSynchronize(stream));
  const auto b = std::chrono::steady_clock::now();
  CC(sim, ccake_check(sim));
  const double sec = std::chrono::duration<double>(b - a).count();
  std::printf("{\"particles\": %lld, \"steps\": %d, \"seconds\": %.6f, \"ms_per_step\": %.6f, "
              "\"particle_steps_per_s\": %.6e}\n",
              (long long)n, steps, sec, sec / steps * 1e3, (double)n * steps / sec);
  CC(sim, ccake_destroy(sim));
  CC(nullptr, ccake_eos_destroy(eos));
  CK(hipStreamDestroy(stream));
  CK(hipFree(ws));
  return 0;
}
