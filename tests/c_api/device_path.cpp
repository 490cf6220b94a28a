// C consumer of the library's device-memory entry points: the result goes to
// a hipMalloc'ed buffer on the caller's stream and must equal the host-result
// entry point's output.  Exit status 0 and "device path ok" on success.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "shatterbc.h"

int main() {
  // a 60-cycle with chords every 7 vertices and three pendants
  const int n = 63;
  std::vector<std::vector<int>> adj(n);
  auto add = [&](int a, int b) {
    adj[a].push_back(b);
    adj[b].push_back(a);
  };
  for (int i = 0; i < 60; ++i) add(i, (i + 1) % 60);
  for (int i = 0; i < 60; i += 7) add(i, (i + 30) % 60);
  add(60, 5);
  add(61, 5);
  add(62, 33);
  std::vector<int32_t> rp(n + 1, 0), col;
  for (int v = 0; v < n; ++v) {
    rp[v + 1] = rp[v] + (int)adj[v].size();
    for (int w : adj[v]) col.push_back(w);
  }
  sbc_context ctx;
  sbc_graph g;
  if (sbc_context_create(0, &ctx) != SBC_OK || sbc_graph_create(n, rp.data(), col.data(), SBC_SANITIZE, &g) != SBC_OK) {
    std::printf("setup failed: %s\n", sbc_last_error());
    return 1;
  }
  std::vector<double> host(n), dev_copy(n);
  if (sbc_betweenness(ctx, g, SBC_COMPRESSED, host.data(), nullptr) != SBC_OK) {
    std::printf("host path failed: %s\n", sbc_last_error());
    return 1;
  }
  double* d = nullptr;
  hipStream_t s;
  if (hipMalloc(&d, sizeof(double) * n) != hipSuccess || hipStreamCreate(&s) != hipSuccess) return 1;
  sbc_run_stats st;
  if (sbc_betweenness_device(ctx, g, SBC_COMPRESSED, d, s, &st) != SBC_OK) {
    std::printf("device path failed: %s\n", sbc_last_error());
    return 1;
  }
  if (hipMemcpy(dev_copy.data(), d, sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess) return 1;
  double worst = 0;
  for (int v = 0; v < n; ++v) {
    const double ref = host[v];
    if (ref == 0) {
      if (dev_copy[v] != 0) {
        std::printf("vertex %d: %g, want 0\n", v, dev_copy[v]);
        return 1;
      }
      continue;
    }
    worst = std::fmax(worst, std::fabs(dev_copy[v] - ref) / ref);
  }
  (void)hipFree(d);
  (void)hipStreamDestroy(s);
  sbc_graph_destroy(g);
  sbc_context_destroy(ctx);
  if (worst > 1e-12) {
    std::printf("max relative difference %g\n", worst);
    return 1;
  }
  std::printf("device path ok (max rel diff %g)\n", worst);
  return 0;
}
