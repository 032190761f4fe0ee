// Host-side planning code of the library under AddressSanitizer and UBSan (built by
// tests/test_host_sanitizers.py): host-only plans of random networks in every precision and
// split policy (describe, step records, cost-model features), sparse-state plans of random
// bitstrings, and the creation error paths.  Prints "ok <plans built>" or a failure code.
#include <cstdio>
#include <cstdlib>
#include <vector>
#include <random>
#include "../../include/tn.h"

static int g_built = 0;

static int run_random(unsigned seed) {
  std::mt19937 rng(seed);
  const int n = 3 + rng() % 12;
  // a random network: labels on pairs of tensors, a few open
  std::vector<std::vector<int32_t>> labels(n);
  std::vector<std::vector<int64_t>> extents(n);
  int next = 0;
  for (int t = 1; t < n; ++t) {            // a tree plus extra bonds
    int u = rng() % t;
    labels[t].push_back(next); labels[u].push_back(next); ++next;
  }
  for (int e = 0; e < n; ++e) {
    int a = rng() % n, b = rng() % n;
    if (a == b) continue;
    labels[a].push_back(next); labels[b].push_back(next); ++next;
  }
  std::vector<int32_t> open;
  for (int t = 0; t < n && open.size() < 3; ++t)
    if (rng() % 3 == 0) { labels[t].push_back(next); open.push_back(next); ++next; }
  std::vector<int32_t> ranks(n);
  std::vector<const int32_t*> lp(n);
  std::vector<const int64_t*> ep(n);
  for (int t = 0; t < n; ++t) {
    extents[t].assign(labels[t].size(), 2);
    ranks[t] = (int32_t)labels[t].size();
    lp[t] = labels[t].data();
    ep[t] = extents[t].data();
  }
  std::vector<int32_t> path;
  for (int s = 1; s < n; ++s) { path.push_back(0); path.push_back(s); }
  std::vector<int32_t> sliced;
  if (next > 2 && rng() % 2) sliced.push_back(0);
  for (int prec = 0; prec < 3; ++prec) {
    tn_options o = {};
    o.struct_size = sizeof(tn_options);
    o.precision = prec;
    o.host_only = 1;
    o.split_policy = (int)(rng() % 3);
    tn_plan p = nullptr;
    tn_status st = tn_plan_create(&p, n, ranks.data(), lp.data(), ep.data(), nullptr, (int)open.size(),
                                  open.data(), n - 1, path.data(), (int)sliced.size(), sliced.data(), &o);
    if (st != TN_OK) { tn_plan_destroy(p); continue; }
    tn_plan_info info;
    if (tn_plan_describe(p, &info) != TN_OK) return 1;
    std::vector<tn_step_info> steps(info.n_steps);
    if (tn_plan_steps(p, steps.data(), info.n_steps) != TN_OK) return 2;
    std::vector<float> f(TN_COST_FEATURES);
    for (int s = 0; s < info.n_steps; ++s)
      if (tn_plan_step_features(p, s, -1, f.data(), TN_COST_FEATURES) != TN_OK) return 3;
    tn_plan_destroy(p);
    ++g_built;
  }
  // the same network as a sparse state: every open label measured on random bitstrings
  if (!open.empty()) {
    const int nb = 1 + (int)(rng() % 40);
    std::vector<uint8_t> bits(nb * open.size());
    for (auto& b : bits) b = (uint8_t)(rng() % 2);
    tn_options o = {};
    o.struct_size = sizeof(tn_options);
    o.precision = (int)(rng() % 3);
    o.host_only = 1;
    tn_plan p = nullptr;
    tn_status st = tn_plan_create_sparse(&p, n, ranks.data(), lp.data(), ep.data(), nullptr, (int)open.size(),
                                         open.data(), n - 1, path.data(), 0, nullptr, nb, bits.data(), &o);
    if (st == TN_OK) {
      std::vector<int64_t> idx(nb);
      if (tn_plan_sparse_index(p, idx.data(), nb) != TN_OK) return 4;
      ++g_built;
    }
    tn_plan_destroy(p);
  }
  return 0;
}

static int run_errors() {
  int32_t ranks[2] = {1, 1};
  int32_t l0[1] = {0}, l1[1] = {1};
  int64_t e0[1] = {2}, e1[1] = {3};
  const int32_t* lp[2] = {l0, l1};
  const int64_t* ep[2] = {e0, e1};
  int32_t path[2] = {0, 1};
  tn_options o = {};
  o.struct_size = sizeof(tn_options);
  o.host_only = 1;
  tn_plan p = nullptr;
  if (tn_plan_create(&p, 2, ranks, lp, ep, nullptr, 0, nullptr, 1, path, 0, nullptr, &o) != TN_E_UNSUPPORTED) return 10;
  if (p) return 11;
  if (tn_plan_create(&p, 0, ranks, lp, ep, nullptr, 0, nullptr, 0, path, 0, nullptr, &o) != TN_E_ARG) return 12;
  e1[0] = 2;
  int32_t bad_path[2] = {0, 0};
  if (tn_plan_create(&p, 2, ranks, lp, ep, nullptr, 0, nullptr, 1, bad_path, 0, nullptr, &o) != TN_E_PATH) return 13;
  tn_plan_destroy(nullptr);
  return 0;
}

int main() {
  int rc = run_errors();
  if (rc) { std::printf("error paths: %d\n", rc); return rc; }
  for (unsigned s = 0; s < 300; ++s) {
    rc = run_random(s);
    if (rc) { std::printf("seed %u: %d\n", s, rc); return rc; }
  }
  std::printf("ok %d\n", g_built);
  return 0;
}
