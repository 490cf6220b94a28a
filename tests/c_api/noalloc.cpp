// C consumer of sbc_piece_bc_noalloc (the entry point that allocates no device
// memory): two calls in a row on device-resident attributed pieces -- a
// larger one, then a smaller one, so the second call finds the first call's
// state in the shared scratch -- each checked against sbc_piece_bc (the host
// entry point with the library's own allocations) to 1e-9 relative, exactly 0
// where that is 0, and device flags 0.  A piece beyond the size limit must be
// refused without running.  Exit status 0 and "noalloc ok" on success.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "shatterbc.h"

struct Piece {
  int n;
  std::vector<int32_t> rp, col, reach, ident;
};

// A random connected piece: a Hamiltonian cycle plus random chords, with
// reach in 1..4 and ident in 1..3.
static Piece make_piece(int n, int chords, unsigned seed) {
  std::mt19937 r(seed);
  std::vector<std::vector<int>> adj(n);
  auto has = [&](int a, int b) {
    for (int x : adj[a])
      if (x == b) return true;
    return false;
  };
  auto add = [&](int a, int b) {
    if (a == b || has(a, b)) return;
    adj[a].push_back(b);
    adj[b].push_back(a);
  };
  for (int i = 0; i < n; ++i) add(i, (i + 1) % n);
  std::uniform_int_distribution<int> pick(0, n - 1);
  for (int k = 0; k < chords; ++k) add(pick(r), pick(r));
  Piece p;
  p.n = n;
  p.rp.assign(n + 1, 0);
  for (int v = 0; v < n; ++v) {
    std::vector<int> nb = adj[v];
    std::sort(nb.begin(), nb.end());
    for (int w : nb) p.col.push_back(w);
    p.rp[v + 1] = (int32_t)p.col.size();
  }
  std::uniform_int_distribution<int> rr(1, 4), kk(1, 3);
  for (int v = 0; v < n; ++v) {
    p.reach.push_back(rr(r));
    p.ident.push_back(kk(r));
  }
  return p;
}

template <typename T>
static T* upload(const std::vector<T>& v) {
  T* d = nullptr;
  if (hipMalloc(&d, sizeof(T) * std::max<size_t>(v.size(), 1)) != hipSuccess) return nullptr;
  if (!v.empty() && hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  return d;
}

static int check(sbc_context ctx, const Piece& p, hipStream_t s, const char* what) {
  std::vector<double> want(p.n), got(p.n);
  if (sbc_piece_bc(ctx, p.n, p.rp.data(), p.col.data(), p.reach.data(), p.ident.data(), 0, want.data(), nullptr) !=
      SBC_OK) {
    std::printf("%s: sbc_piece_bc failed: %s\n", what, sbc_last_error());
    return 1;
  }
  int32_t *drp = upload(p.rp), *dcol = upload(p.col), *dre = upload(p.reach), *did = upload(p.ident);
  double* dbc = nullptr;
  int32_t* dflags = nullptr;
  if (!drp || !dcol || !dre || !did || hipMalloc(&dbc, sizeof(double) * p.n) != hipSuccess ||
      hipMalloc(&dflags, sizeof(int32_t)) != hipSuccess) {
    std::printf("%s: test setup allocation failed\n", what);
    return 1;
  }
  const int32_t arcs = (int32_t)p.col.size();
  if (sbc_piece_bc_noalloc(ctx, p.n, arcs, drp, dcol, dre, did, dbc, dflags, s) != SBC_OK) {
    std::printf("%s: sbc_piece_bc_noalloc failed: %s\n", what, sbc_last_error());
    return 1;
  }
  int32_t flags = -1;
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(got.data(), dbc, sizeof(double) * p.n, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&flags, dflags, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) {
    std::printf("%s: copy back failed\n", what);
    return 1;
  }
  double worst = 0;
  for (int v = 0; v < p.n; ++v) {
    if (want[v] == 0) {
      if (got[v] != 0) {
        std::printf("%s: vertex %d is %g, want 0\n", what, v, got[v]);
        return 1;
      }
      continue;
    }
    worst = std::fmax(worst, std::fabs(got[v] - want[v]) / std::fabs(want[v]));
  }
  (void)hipFree(drp);
  (void)hipFree(dcol);
  (void)hipFree(dre);
  (void)hipFree(did);
  (void)hipFree(dbc);
  (void)hipFree(dflags);
  std::printf("%s: n=%d arcs=%d flags=%d max rel diff %g\n", what, p.n, arcs, flags, worst);
  if (flags != 0 || worst > 1e-9) return 1;
  return 0;
}

int main() {
  sbc_context ctx;
  if (sbc_context_create(0, &ctx) != SBC_OK) {
    std::printf("context: %s\n", sbc_last_error());
    return 1;
  }
  hipStream_t s;
  if (hipStreamCreate(&s) != hipSuccess) return 1;
  const Piece big = make_piece(2500, 5000, 7), small = make_piece(300, 400, 11);
  if (check(ctx, big, s, "first call") || check(ctx, small, s, "second call, smaller")) return 1;
  // beyond the limit: refused before anything runs
  int32_t* none = nullptr;
  if (hipMalloc(&none, 64) != hipSuccess) return 1;
  const sbc_status rc = sbc_piece_bc_noalloc(ctx, SBC_NOALLOC_MAX_VERTICES + 1, 0, none, none, nullptr, nullptr,
                                             reinterpret_cast<double*>(none), nullptr, s);
  if (rc != SBC_E_TOO_LARGE) {
    std::printf("oversized piece: status %d, want SBC_E_TOO_LARGE\n", rc);
    return 1;
  }
  (void)hipFree(none);
  (void)hipStreamDestroy(s);
  sbc_context_destroy(ctx);
  std::printf("noalloc ok\n");
  return 0;
}
