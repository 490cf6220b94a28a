// C consumer of the library's device-memory entry points: the result goes to
// a hipMalloc'ed buffer on the caller's stream.  Both it and the host-result
// entry point's output must equal the oracle's values for the same graph
// (tests/golden/device_path_bc.txt, written by the script beside it from the
// oracle alone) within 1e-9 relative, and exactly 0 where those are 0.
// Run from the repository root.  Exit status 0 and "device path ok" on success.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "shatterbc.h"

// Reads the golden file: a comment line, the vertex count, one value per line.
static bool read_golden(const char* path, std::vector<double>* out) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  if (!std::fgets(line, sizeof line, f)) {
    std::fclose(f);
    return false;
  }
  int n = 0;
  if (std::fscanf(f, "%d", &n) != 1 || n <= 0) {
    std::fclose(f);
    return false;
  }
  out->resize(n);
  for (int i = 0; i < n; ++i)
    if (std::fscanf(f, "%lf", &(*out)[i]) != 1) {
      std::fclose(f);
      return false;
    }
  std::fclose(f);
  return true;
}

// Largest relative difference from the golden values; -1 on a nonzero value
// where the golden value is 0.
static double worst_rel(const std::vector<double>& got, const std::vector<double>& want, const char* what) {
  double worst = 0;
  for (size_t v = 0; v < want.size(); ++v) {
    if (want[v] == 0) {
      if (got[v] != 0) {
        std::printf("%s: vertex %zu is %g, oracle 0\n", what, v, got[v]);
        return -1;
      }
      continue;
    }
    worst = std::fmax(worst, std::fabs(got[v] - want[v]) / std::fabs(want[v]));
  }
  return worst;
}

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
  std::vector<double> want;
  if (!read_golden("tests/golden/device_path_bc.txt", &want) || (int)want.size() != n) {
    std::printf("cannot read tests/golden/device_path_bc.txt (run from the repository root)\n");
    return 1;
  }
  const double wh = worst_rel(host, want, "host output");
  const double wd = worst_rel(dev_copy, want, "device output");
  (void)hipFree(d);
  (void)hipStreamDestroy(s);
  sbc_graph_destroy(g);
  sbc_context_destroy(ctx);
  if (wh < 0 || wd < 0 || wh > 1e-9 || wd > 1e-9) {
    std::printf("max relative difference from the oracle: host %g, device %g\n", wh, wd);
    return 1;
  }
  std::printf("device path ok (max rel diff from the oracle: host %g, device %g)\n", wh, wd);
  return 0;
}
