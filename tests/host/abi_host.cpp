// Host-side checks of the C-ABI library: argument validation of every entry point, the launch
// plan's layout of a batch into drop descriptors and work items, the user-group virtual drops of
// drops with more than 64 users, and the Gauss-Legendre table the context uploads.  Built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host code; no kernel runs.  The library
// source is included so that its internal helpers are callable; the kernels it refers to come
// from the built library.  A context object is constructed directly, so without a GPU every call
// that passes validation stops at its first device call (XLMIMO_EDEVICE).
#include "api.cpp"

#include <cstdio>
#include <cstdlib>
#include <random>

namespace {

int g_fail = 0, g_checks = 0;
#define CHECK(cond)                                                               \
  do {                                                                            \
    ++g_checks;                                                                   \
    if (!(cond)) {                                                                \
      std::fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);        \
      ++g_fail;                                                                   \
    }                                                                             \
  } while (0)

xlmimo_array make_array(int geom, int64_t ny, int64_t nz) {
  xlmimo_array a{};
  a.geometry = geom;
  a.amp_model = XLMIMO_AMP_FREESPACE;
  a.n_y = ny;
  a.n_z = nz;
  a.spacing_m = 5.355e-3;
  a.wavelength_m = 10.71e-3;
  a.beta0 = 1.0;
  return a;
}

void test_check_array() {
  xlmimo_ctx c;
  xlmimo_array a = make_array(XLMIMO_ULA, 256, 1);
  CHECK(check_array(&c, &a) == XLMIMO_OK);
  a = make_array(XLMIMO_UPA, 512, 512);
  CHECK(check_array(&c, &a) == XLMIMO_OK);
  CHECK(check_array(&c, nullptr) == XLMIMO_EINVAL);
  struct Bad {
    const char* what;
    void (*edit)(xlmimo_array&);
  };
  const Bad bad[] = {
      {"geometry", [](xlmimo_array& x) { x.geometry = 7; }},
      {"amplitude model", [](xlmimo_array& x) { x.amp_model = -1; }},
      {"spacing 0", [](xlmimo_array& x) { x.spacing_m = 0.0; }},
      {"spacing NaN", [](xlmimo_array& x) { x.spacing_m = std::nan(""); }},
      {"wavelength inf", [](xlmimo_array& x) { x.wavelength_m = INFINITY; }},
      {"PNUSW beta0 0", [](xlmimo_array& x) { x.amp_model = XLMIMO_AMP_PNUSW; x.beta0 = 0.0; }},
      {"n_y 0", [](xlmimo_array& x) { x.n_y = 0; }},
      {"n_z negative", [](xlmimo_array& x) { x.n_z = -3; }},
      {"2^31 elements", [](xlmimo_array& x) { x.n_y = 65536; x.n_z = 32768; }},
      // a product that wraps around int64 must not pass as a small panel
      {"2^64 elements", [](xlmimo_array& x) { x.n_y = int64_t(1) << 33; x.n_z = int64_t(1) << 31; }},
      {"huge n_y", [](xlmimo_array& x) { x.n_y = INT64_MAX; x.n_z = INT64_MAX; }},
  };
  for (const Bad& b : bad) {
    xlmimo_array x = make_array(XLMIMO_UPA, 64, 64);
    b.edit(x);
    const int rc = check_array(&c, &x);
    if (rc != XLMIMO_EINVAL) std::fprintf(stderr, "array case '%s' gave %d\n", b.what, rc);
    CHECK(rc == XLMIMO_EINVAL);
    CHECK(!c.err.empty());
  }
  xlmimo_array u = make_array(XLMIMO_ULA, 256, 2);   // a ULA has one row
  CHECK(check_array(&c, &u) == XLMIMO_EINVAL);
}

void test_check_batch() {
  xlmimo_ctx c;
  const int32_t k_ok[3] = {1, 16, 64};
  const int64_t n_ok[3] = {1, 1000, 2147483647LL};
  const double pos = 0.0;
  xlmimo_batch b{3, n_ok, k_ok, &pos};
  CHECK(check_batch(&c, &b, true) == XLMIMO_OK);
  CHECK(check_batch(&c, nullptr, true) == XLMIMO_EINVAL);
  xlmimo_batch empty{0, nullptr, nullptr, nullptr};
  CHECK(check_batch(&c, &empty, true) == XLMIMO_OK);   // no drops: nothing else is read
  xlmimo_batch neg{-1, n_ok, k_ok, &pos};
  CHECK(check_batch(&c, &neg, true) == XLMIMO_EINVAL);
  xlmimo_batch big{int64_t(1) << 31, n_ok, k_ok, &pos};
  CHECK(check_batch(&c, &big, true) == XLMIMO_EINVAL);
  xlmimo_batch no_k{3, n_ok, nullptr, &pos};
  CHECK(check_batch(&c, &no_k, true) == XLMIMO_EINVAL);
  xlmimo_batch no_pos{3, n_ok, k_ok, nullptr};
  CHECK(check_batch(&c, &no_pos, true) == XLMIMO_EINVAL);
  CHECK(check_batch(&c, &no_pos, false) == XLMIMO_OK);
  const int32_t k_bad[4][3] = {{0, 1, 1}, {1, 65, 1}, {1, 1, -5}, {1, 1, INT32_MAX}};
  for (const auto& kb : k_bad) {
    xlmimo_batch x{3, n_ok, kb, &pos};
    CHECK(check_batch(&c, &x, true) == XLMIMO_EINVAL);
  }
  const int32_t k_1000[3] = {1000, 1024, 2};
  xlmimo_batch wide{3, n_ok, k_1000, &pos};
  CHECK(check_batch(&c, &wide, true) == XLMIMO_EINVAL);
  CHECK(check_batch(&c, &wide, true, XLMIMO_MAX_USERS_EXACT) == XLMIMO_OK);
  const int64_t n_bad[3][3] = {{0, 1, 1}, {1, -1, 1}, {1, 1, 2147483648LL}};
  for (const auto& nb : n_bad) {
    xlmimo_batch x{3, nb, k_ok, &pos};
    CHECK(check_batch(&c, &x, true) == XLMIMO_EINVAL);
  }
}

void test_chunk_length() {
  const int64_t totals[] = {0, 1, 255, 2048, 100000, 262144LL * 10000, INT64_MAX / 2};
  const int grids[] = {-5, 0, 1, 7, 256, 1024, 1 << 20};
  for (int64_t t : totals)
    for (int g : grids) {
      const int64_t ch = chunk_length(t, g);
      CHECK(ch % 256 == 0);
      CHECK(ch >= 2048 && ch <= 65536);
    }
}

// The plan layout of a batch: every drop's elements covered once by its items, offsets that are
// the prefix sums of its users, Gram entries, user pairs and partial images, and the longest-first
// item order.
void check_layout(int n, const std::vector<int64_t>& ne, const std::vector<int32_t>& kk, int64_t ch) {
  HostLayout L;
  layout_drops(n, ne.data(), kk.data(), nullptr, L);
  layout_items(ch, L);
  int64_t users = 0, gram = 0, pairs = 0, parts = 0, elems = 0;
  std::vector<int64_t> covered(n, 0);
  std::vector<std::vector<char>> seen(n);
  for (int d = 0; d < n; ++d) {
    const DropK& dk = L.drops[d];
    CHECK(dk.user_off == users && dk.gram_off == gram && dk.pair_off == pairs && dk.part_off == parts);
    CHECK(dk.k == kk[d] && dk.n_elems == ne[d] && dk.nb == (kk[d] + 15) / 16 && dk.cross == 0);
    CHECK(dk.n_items == (ne[d] + ch - 1) / ch);
    users += kk[d];
    gram += (int64_t)kk[d] * kk[d];
    pairs += (int64_t)kk[d] * (kk[d] - 1) / 2;
    parts += (int64_t)dk.n_items * partial_values(dk.nb) * 64;
    elems += ne[d];
    seen[d].assign(dk.n_items, 0);
  }
  CHECK(L.total_users == users && L.gram_elems == gram && L.n_pairs == pairs && L.partial_doubles == parts);
  CHECK(L.total_elems == elems);
  int64_t prev_cost = INT64_MAX;
  for (const ItemK& it : L.items) {
    CHECK(it.drop >= 0 && it.drop < n);
    if (it.drop < 0 || it.drop >= n) continue;
    const DropK& dk = L.drops[it.drop];
    CHECK(it.chunk >= 0 && it.chunk < dk.n_items);
    if (it.chunk < 0 || it.chunk >= dk.n_items) continue;
    CHECK(!seen[it.drop][it.chunk]);
    seen[it.drop][it.chunk] = 1;
    CHECK(it.e_begin == (int64_t)it.chunk * ch);
    CHECK(it.e_end > it.e_begin && it.e_end <= dk.n_elems && it.e_end - it.e_begin <= ch);
    covered[it.drop] += it.e_end - it.e_begin;
    const int nb = dk.nb;
    const int64_t cost = (int64_t)(it.e_end - it.e_begin) * (nb * 8 + 3 * (nb * (nb + 1) / 2 + nb * nb));
    CHECK(cost <= prev_cost);
    prev_cost = cost;
  }
  for (int d = 0; d < n; ++d) CHECK(covered[d] == ne[d]);
}

void test_layout() {
  std::mt19937_64 rng(20250318);
  for (int rep = 0; rep < 40; ++rep) {
    const int n = 1 + (int)(rng() % 300);
    std::vector<int64_t> ne(n);
    std::vector<int32_t> kk(n);
    for (int d = 0; d < n; ++d) {
      ne[d] = 1 + (int64_t)(rng() % (rep % 4 == 0 ? 300000 : 5000));
      kk[d] = 1 + (int32_t)(rng() % 64);
    }
    const int64_t ch = chunk_length(rng() % 100000000, 1 + (int)(rng() % 2048));
    check_layout(n, ne, kk, ch);
  }
  // the largest element count a drop may have, in the shortest chunks
  check_layout(2, {2147483647LL, 1}, {64, 1}, 2048);
  HostLayout L;
  layout_drops(0, nullptr, nullptr, nullptr, L);
  layout_items(2048, L);
  CHECK(L.items.empty() && L.partial_doubles == 0);
}

// Entry points given a NULL context, NULL handles or invalid arguments with a constructed
// context: an error code, never a crash, and no device call before validation.
void test_entry_points() {
  CHECK(xlmimo_gram_exact(nullptr, nullptr, nullptr, 0, nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_gram_exact_noalloc(nullptr, nullptr, nullptr, 0, nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_gram_update_users(nullptr, nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_cholesky(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_cholesky_update_users(nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                                     nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_gram_closedform(nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_zf_mmse_sumrate(nullptr, nullptr, nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr, nullptr) ==
        XLMIMO_EINVAL);
  CHECK(xlmimo_capacity_sweep(nullptr, nullptr, 0, nullptr, nullptr, 0, nullptr, 0.0, 0, nullptr, 0, 0.0, 0.0,
                              nullptr, nullptr, nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_mlp_create(nullptr, 256, 4, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_mlp_destroy(nullptr) == XLMIMO_OK);
  CHECK(xlmimo_mlp_param_count(nullptr) == -1);
  CHECK(xlmimo_mlp_set_params(nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_mlp_get_params(nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_mlp_set_gate(nullptr, 0, nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_mlp_pair_inputs(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                               nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_mlp_loss_grad(nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
        XLMIMO_EINVAL);
  CHECK(xlmimo_mlp_train_step(nullptr, nullptr, 0, nullptr, nullptr, nullptr, 0.f, nullptr, nullptr) ==
        XLMIMO_EINVAL);
  CHECK(xlmimo_mlp_train(nullptr, nullptr, 0, nullptr, nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr) ==
        XLMIMO_EINVAL);
  CHECK(xlmimo_mlp_forward(nullptr, nullptr, 0, nullptr, nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_gram_closedform_mlp(nullptr, nullptr, nullptr, 0, nullptr, 0.0, nullptr, nullptr, nullptr) ==
        XLMIMO_EINVAL);
  CHECK(xlmimo_graph_begin(nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_graph_end(nullptr, nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_graph_launch(nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_graph_node_count(nullptr) == -1);
  CHECK(xlmimo_graph_destroy(nullptr) == XLMIMO_OK);
  CHECK(xlmimo_autotune_exact(nullptr, nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_timing_enable(nullptr, 1) == XLMIMO_EINVAL);
  CHECK(xlmimo_timing_read(nullptr, nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_ctx_destroy(nullptr) == XLMIMO_OK);
  CHECK(xlmimo_ctx_create(nullptr, 0) == XLMIMO_EINVAL);
  CHECK(std::strcmp(xlmimo_last_error(nullptr), "no context") == 0);
  CHECK(std::strncmp(xlmimo_version(), "xlmimo", 6) == 0);

  const int32_t k3[3] = {2, 16, 40};
  xlmimo_batch b3{3, nullptr, k3, nullptr};
  CHECK(xlmimo_pair_count(&b3) == 1 + 120 + 780);
  CHECK(xlmimo_pair_count(nullptr) == -1);
  xlmimo_batch nok{2, nullptr, nullptr, nullptr};
  CHECK(xlmimo_pair_count(&nok) == -1);

  // validation with a constructed context: the messages name the argument; nothing reaches the device
  xlmimo_ctx c;
  xlmimo_array a = make_array(XLMIMO_ULA, 256, 1);
  const double pos[3 * 16] = {};
  const int32_t k1[1] = {16};
  xlmimo_batch b{1, nullptr, k1, pos};
  double out[2 * 256];
  CHECK(xlmimo_gram_exact(&c, &a, &b, 9, out, nullptr) == XLMIMO_EINVAL);
  CHECK(c.err.find("precision") != std::string::npos);
  CHECK(xlmimo_gram_exact(&c, &a, &b, XLMIMO_FP64, nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(c.err.find("gram_out") != std::string::npos);
  xlmimo_batch b0{0, nullptr, nullptr, nullptr};
  CHECK(xlmimo_gram_exact(&c, &a, &b0, XLMIMO_FP64, nullptr, nullptr) == XLMIMO_OK);   // no drops: no-op
  xlmimo_array bad = make_array(XLMIMO_ULA, 0, 1);
  CHECK(xlmimo_gram_closedform(&c, &bad, &b, XLMIMO_CF_UNIFORM, out, nullptr, nullptr) == XLMIMO_EINVAL);
  CHECK(xlmimo_timing_read(&c, nullptr, nullptr) == XLMIMO_EINVAL);
  // a capture in progress refuses other streams and the calls that cannot be captured
  c.capturing = true;
  c.cap_stream = reinterpret_cast<hipStream_t>(0x10);
  CHECK(xlmimo_gram_exact(&c, &a, &b, XLMIMO_FP64, out, nullptr) == XLMIMO_EINVAL);
  CHECK(c.cap_failed);
  c.capturing = false;
  c.cap_failed = false;
}

// The user-group plan of one drop: every user pair (i < j) computed by exactly one virtual drop
// that copies it out (its cross block, or the own block of its group), every group's own block
// copied exactly once, cross-only drops exactly the pairs that copy no own block, and at most 64
// users per virtual drop.
void test_group_pairs() {
  for (int K : {1, 2, 31, 63, 64, 65, 96, 97, 128, 200, 511, 1000, 1024}) {
    const std::vector<GroupPair> gps = group_pairs(K);
    std::vector<int> seen((size_t)K * K, 0);
    for (const GroupPair& gp : gps) {
      CHECK(gp.ka >= 1 && gp.kb >= 0 && gp.ka + gp.kb <= XLMIMO_MAX_USERS);
      CHECK(gp.a0 >= 0 && gp.a0 + gp.ka <= K && gp.b0 >= 0 && gp.b0 + gp.kb <= K);
      CHECK(gp.cross == ((gp.flags & (kVCopyA | kVCopyB)) == 0 ? 1 : 0) || K <= XLMIMO_MAX_USERS);
      if (gp.kb > 0) CHECK(gp.a0 + gp.ka <= gp.b0);   // disjoint groups, a before b
      for (int i = 0; i < gp.ka; ++i)
        for (int j = 0; j < gp.kb; ++j) ++seen[(size_t)(gp.a0 + i) * K + (gp.b0 + j)];
      auto own = [&](int o, int k) {
        for (int i = 0; i < k; ++i)
          for (int j = i + 1; j < k; ++j) ++seen[(size_t)(o + i) * K + (o + j)];
      };
      if (gp.flags & kVCopyA) own(gp.a0, gp.ka);
      if (gp.flags & kVCopyB) own(gp.b0, gp.kb);
    }
    int bad = 0;
    for (int i = 0; i < K; ++i)
      for (int j = i + 1; j < K; ++j) bad += seen[(size_t)i * K + j] != 1;
    if (bad) std::fprintf(stderr, "K = %d: %d user pairs not covered exactly once\n", K, bad);
    CHECK(bad == 0);
    const int g = (K + kGroupUsers - 1) / kGroupUsers;
    CHECK((int)gps.size() == (K <= XLMIMO_MAX_USERS ? 1 : g * (g - 1) / 2));
  }
}

// Launch plans built against a constructed context: the host layout runs in full (the drops,
// the items and, above 64 users, the user-group virtual drops) and the build stops cleanly at
// the first device allocation when no GPU is present.
void test_plan_builds() {
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess) n_dev = 0;
  (void)hipGetLastError();
  if (n_dev > 0) return;   // with a device the plans would be uploaded: that is the GPU tests' part
  xlmimo_ctx c;
  xlmimo_array a = make_array(XLMIMO_ULA, 65536, 1);
  const int32_t kk[4] = {16, 64, 1000, 3};
  const int64_t ne[4] = {4096, 70001, 65536, 1};
  xlmimo_batch b{4, ne, kk, nullptr};
  Plan* p = nullptr;
  CHECK(get_plan(&c, &a, &b, nullptr, &p) == XLMIMO_EDEVICE);
  CHECK(c.plans.empty());
  Plan q;
  q.n_drops = 4;
  q.k_max = 1000;
  q.ne_host.assign(ne, ne + 4);
  q.k_host.assign(kk, kk + 4);
  CHECK(build_groups(&c, &a, q) == XLMIMO_EDEVICE);
  CHECK(q.vplan == nullptr);
  xlmimo_ctx* made = reinterpret_cast<xlmimo_ctx*>(0x1);
  CHECK(xlmimo_ctx_create(&made, 0) == XLMIMO_EDEVICE);
  CHECK(made == nullptr);
}

// The Gauss-Legendre rule the context uploads: weights summing to 2, nodes symmetric in (-1, 1),
// and exact integration of x^(2n-2) (degree 2n - 1 is the rule's reach).
void test_gauss_legendre() {
  for (int n : {1, 2, 7, 64, 200}) {
    std::vector<double> t;
    gauss_legendre(n, t);
    CHECK((int)t.size() == 2 * n);
    double wsum = 0.0, mom = 0.0;
    for (int i = 0; i < n; ++i) {
      const double x = t[2 * i], w = t[2 * i + 1];
      CHECK(x > -1.0 && x < 1.0 && w > 0.0);
      wsum += w;
      mom += w * std::pow(x, 2 * n - 2);
    }
    CHECK(std::fabs(wsum - 2.0) < 1e-13);
    CHECK(std::fabs(mom - 2.0 / (2 * n - 1)) < 1e-12);
  }
}

}  // namespace

int main() {
  test_check_array();
  test_check_batch();
  test_chunk_length();
  test_layout();
  test_group_pairs();
  test_entry_points();
  test_plan_builds();
  test_gauss_legendre();
  std::printf("host checks: %d of %d passed\n", g_checks - g_fail, g_checks);
  return g_fail == 0 ? 0 : 1;
}
