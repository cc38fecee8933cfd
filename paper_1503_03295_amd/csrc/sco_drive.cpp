// sco_drive.cpp -- native driver of libsco through its C ABI only (no Python, no
// torch): one chain on a periodic or open lattice, `warmup` steps, then `steps`
// timed steps as one sco_run, then `split` steps as separate switch / colour / sweep
// launches with their phase times.  Used for profiling the kernels with rocprofv3
// and as a minimal example of the library's calling sequence.
//
//   sco_drive L periodic T kappa n_sw warmup steps split
#include <hip/hip_runtime.h>

#include <link.h>

#include <cstdio>
#include <cstdlib>

#include "../../include/sco.h"

#define HIP_OK(expr)                                      \
  do {                                                    \
    if ((expr) != hipSuccess) return die(#expr, SCO_EHIP); \
  } while (0)

static int die(const char* what, int rc) {
  std::fprintf(stderr, "sco_drive: %s failed: %s (%d)\n", what, sco_strerror(rc), rc);
  return 1;
}

// The address range of every loaded library, on stderr: a fault reported at exit
// (by a profiler's handler, as raw addresses) can then be put down to a library.
static int print_range(dl_phdr_info* info, size_t, void*) {
  uintptr_t lo = UINTPTR_MAX, hi = 0;
  for (int i = 0; i < info->dlpi_phnum; ++i) {
    const ElfW(Phdr)& ph = info->dlpi_phdr[i];
    if (ph.p_type != PT_LOAD) continue;
    const uintptr_t b = info->dlpi_addr + ph.p_vaddr;
    if (b < lo) lo = b;
    if (b + ph.p_memsz > hi) hi = b + ph.p_memsz;
  }
  if (hi > lo) std::fprintf(stderr, "library %#zx-%#zx %s\n", static_cast<size_t>(lo), static_cast<size_t>(hi),
                            info->dlpi_name[0] ? info->dlpi_name : "(main)");
  return 0;
}

int main(int argc, char** argv) {
  if (argc != 9) {
    std::fprintf(stderr, "usage: %s L periodic T kappa n_sw warmup steps split\n", argv[0]);
    return 2;
  }
  sco_chain_params p{};
  p.L = std::atoi(argv[1]);
  p.periodic = std::atoi(argv[2]);
  p.n_images = 8;
  p.n_sw = std::atoi(argv[5]);
  p.J = 1.0;
  p.D = 0.1;
  p.T = std::atof(argv[3]);
  p.kappa = std::atof(argv[4]);
  p.seed = 1;
  p.chain_id = 0;
  const int warmup = std::atoi(argv[6]), steps = std::atoi(argv[7]), split = std::atoi(argv[8]);
  if (warmup < 0 || steps < 1 || split < 0) return 2;

  size_t bytes = 0;
  int rc = sco_workspace_size(&p, 1, &bytes);
  if (rc) return die("sco_workspace_size", rc);
  void* ws = nullptr;
  if (hipMalloc(&ws, bytes) != hipSuccess) return die("hipMalloc", SCO_EHIP);
  hipStream_t s;
  if (hipStreamCreate(&s) != hipSuccess) return die("hipStreamCreate", SCO_EHIP);
  sco_ctx* ctx = nullptr;
  rc = sco_init(&ctx, &p, 1, ws, bytes, nullptr, s);
  if (rc) return die("sco_init", rc);
  std::printf("L=%d periodic=%d T=%g kappa=%g n_sw=%d workspace=%.1f MB\n", p.L, p.periodic, p.T, p.kappa,
              p.n_sw, bytes / 1e6);
  std::fflush(stdout);

  // a plain device copy of known size, for scaling memory counters read around it
  {
    const size_t cb = static_cast<size_t>(256) << 20;
    void *src = nullptr, *dst = nullptr;
    HIP_OK(hipMalloc(&src, cb));
    HIP_OK(hipMalloc(&dst, cb));
    HIP_OK(hipMemsetAsync(src, 1, cb, s));
    HIP_OK(hipMemcpyAsync(dst, src, cb, hipMemcpyDeviceToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    HIP_OK(hipFree(src));
    HIP_OK(hipFree(dst));
    std::printf("calibration copy: %zu bytes read and written\n", cb);
  }
  if ((rc = sco_run(ctx, 0, warmup))) return die("sco_run", rc);
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  HIP_OK(hipEventRecord(e0, s));
  if ((rc = sco_run(ctx, warmup, steps))) return die("sco_run", rc);
  HIP_OK(hipEventRecord(e1, s));
  HIP_OK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, e0, e1));
  const double N = static_cast<double>(p.L) * p.L;
  std::printf("timed %d steps: %.4f ms/step, %.4g attempts/s\n", steps, ms / steps,
              N * p.n_sw * steps / (ms * 1e-3));
  std::fflush(stdout);

  double acc[3] = {0, 0, 0};
  for (int t = 0; t < split; ++t) {
    const uint64_t step = static_cast<uint64_t>(warmup + steps + t);
    if ((rc = sco_switch(ctx, step))) return die("sco_switch", rc);
    if ((rc = sco_color(ctx))) return die("sco_color", rc);
    if ((rc = sco_sweep(ctx, step, p.n_sw))) return die("sco_sweep", rc);
    float ph[3];
    if ((rc = sco_phase_times(ctx, ph))) return die("sco_phase_times", rc);
    for (int i = 0; i < 3; ++i) acc[i] += ph[i];
  }
  if (split > 0)
    std::printf("split phases (ms): switch %.4f colour %.4f sweep %.4f\n", acc[0] / split, acc[1] / split,
                acc[2] / split);
  sco_obs o{};
  if ((rc = sco_observables(ctx, &o))) return die("sco_observables", rc);
  std::printf("E=%.10g M=%lld bonds=%lld q=%d kw_rounds=%lld accepted=%lld flags=%lld\n", o.E,
              static_cast<long long>(o.M), static_cast<long long>(o.n_edges), o.q,
              static_cast<long long>(o.kw_rounds), static_cast<long long>(o.accepted),
              static_cast<long long>(o.flags));
  sco_destroy(ctx);
  HIP_OK(hipEventDestroy(e0));
  HIP_OK(hipEventDestroy(e1));
  HIP_OK(hipStreamDestroy(s));
  HIP_OK(hipFree(ws));
  std::fflush(stdout);
  dl_iterate_phdr(print_range, nullptr);
  std::fflush(stderr);
  return 0;
}
