// C ABI of libxlmimo: argument validation, per-context workspace, launch
// plans (work lists) cached per batch shape, and stream-ordered launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "xlmimo.h"

using namespace xl;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
};

struct Plan {
  int n_drops = 0;
  int n_items = 0;
  int nb_max = 1;
  int k_max = 1;
  int64_t total_users = 0;
  int64_t gram_elems = 0;    // complex elements of the whole Gram output
  int64_t n_pairs = 0;       // user pairs i < j over all drops
  int64_t partial_doubles = 0;
  int grid_fp32 = 0, grid_fp64 = 0, grid_fp32h = 0;
  int64_t chunk = 0;         // work-item length in elements
  uint64_t key = 0;          // plan_key of the batch shape
  DropK* d_drops = nullptr;
  ItemK* d_items = nullptr;
  // K > XLMIMO_MAX_USERS: the exact Gram runs over group-pair virtual drops,
  // whose plan is built on the first exact-Gram call of this shape
  std::vector<int64_t> ne_host;   // per-drop N and K, kept only for that build
  std::vector<int32_t> k_host;
  struct Plan* vplan = nullptr;   // owned
  int n_v = 0;
  int64_t n_vusers = 0;
  VDropK* d_v = nullptr;
  int64_t* d_vmap = nullptr;
  VRowK* d_vr = nullptr;          // row plans (moved users): one descriptor per virtual drop
  int n_vr = 0;
  int32_t* d_mdrop = nullptr;     // row plans: drops with moved users, offsets into the drop-local
  int32_t* d_moff = nullptr;      // indices of their moved users (ascending)
  int32_t* d_mloc = nullptr;
  int n_mdrop = 0;
};

}  // namespace

struct xlmimo_ctx {
  int device = 0;
  std::mutex mu;
  std::string err;
  int* d_counter = nullptr;
  double* d_gl = nullptr;  // Gauss-Legendre (node, weight) pairs: the n_gl-node rule, then kFresnelNodes nodes
  int n_gl = 0;
  DevBuf partials, scratch_gram, scratch_gram2, scratch_rates, scratch_bounds, scratch_nlist, scratch_pairs;
  DevBuf scratch_routes;   // per-pair route words of the ULA closed forms UNIFORM and GATED_QUAD
  DevBuf scratch_vpos, scratch_vgram;  // virtual drops of the exact Gram (K > XLMIMO_MAX_USERS)
  DevBuf scratch_work;     // matrices of the workgroup-per-drop rate kernel (K > XLMIMO_MAX_USERS)
  std::vector<double> nlist_host;  // N list last uploaded to scratch_nlist
  std::unordered_map<uint64_t, Plan> plans;
  std::unordered_map<uint64_t, Plan> row_plans;   // moved-user row plans, evicted on their own
  // kernel timing (xlmimo_timing_enable / xlmimo_timing_read)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  // graph capture (xlmimo_graph_*): while any graph of this context exists, device
  // buffers it may reference are retired (freed with the context) instead of freed
  bool capturing = false;
  bool cap_failed = false;
  hipStream_t cap_stream = nullptr;
  int graphs = 0;
  std::vector<void*> retired;
  // autotuned exact-Gram launch shapes (xlmimo_autotune_exact), keyed by plan
  std::unordered_map<uint64_t, int64_t> tuned_chunk;
  std::unordered_map<uint64_t, int> tuned_grid;   // key ^ precision
  hipError_t scratch_init = hipSuccess;   // look-up of the allocation-free path's static array
};

struct xlmimo_graph {
  xlmimo_ctx* ctx = nullptr;
  hipGraphExec_t exec = nullptr;
  size_t n_nodes = 0;
};

namespace {

int set_err(xlmimo_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) {
    c->err = buf;
    if (c->capturing) c->cap_failed = true;  // the graph being captured is incomplete
  }
  return code;
}

#define HIP_TRY(ctx, expr)                                                                               \
  do {                                                                                                   \
    hipError_t e_ = (expr);                                                                              \
    if (e_ != hipSuccess) return set_err((ctx), XLMIMO_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Free device memory that a live graph of the context might still reference.
int release(xlmimo_ctx* c, void* p) {
  if (!p) return XLMIMO_OK;
  if (c->graphs > 0) {
    c->retired.push_back(p);
    return XLMIMO_OK;
  }
  HIP_TRY(c, hipFree(p));
  return XLMIMO_OK;
}

int ensure(xlmimo_ctx* c, DevBuf& b, size_t bytes, hipStream_t s) {
  if (b.n >= bytes) return XLMIMO_OK;
  if (c->capturing)
    return set_err(c, XLMIMO_EINVAL, "workspace must grow to %zu bytes during graph capture: "
                   "run the same calls once before capturing them", bytes);
  if (b.p) {
    HIP_TRY(c, hipStreamSynchronize(s));
    int rc = release(c, b.p);
    if (rc) return rc;
    b.p = nullptr;
    b.n = 0;
  }
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return set_err(c, XLMIMO_ENOMEM, "workspace allocation of %zu bytes failed", bytes);
  }
  b.n = bytes;
  return XLMIMO_OK;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n from the
// Chebyshev initial guess), used by the UPA free-space closed-form diagonal, the
// aperture quadrature and the Fresnel integrals of the closed forms.
void gauss_legendre(int n, std::vector<double>& out) {
  out.assign(2 * n, 0.0);
  const double pi = 3.14159265358979323846264338327950288;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    out[2 * i] = x;
    out[2 * i + 1] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int check_array(xlmimo_ctx* c, const xlmimo_array* a) {
  if (!a) return set_err(c, XLMIMO_EINVAL, "array is NULL");
  if (a->geometry != XLMIMO_ULA && a->geometry != XLMIMO_UPA) return set_err(c, XLMIMO_EINVAL, "bad geometry %d", a->geometry);
  if (a->amp_model != XLMIMO_AMP_FREESPACE && a->amp_model != XLMIMO_AMP_PNUSW)
    return set_err(c, XLMIMO_EINVAL, "bad amplitude model %d", a->amp_model);
  if (!finite_pos(a->spacing_m)) return set_err(c, XLMIMO_EINVAL, "spacing must be finite and > 0");
  if (!finite_pos(a->wavelength_m)) return set_err(c, XLMIMO_EINVAL, "wavelength must be finite and > 0");
  if (a->amp_model == XLMIMO_AMP_PNUSW && !finite_pos(a->beta0)) return set_err(c, XLMIMO_EINVAL, "beta0 must be finite and > 0");
  if (a->n_y < 1 || a->n_z < 1) return set_err(c, XLMIMO_EINVAL, "array sizes must be >= 1");
  if (a->geometry == XLMIMO_ULA && a->n_z != 1) return set_err(c, XLMIMO_EINVAL, "a ULA has n_z == 1");
  if (a->n_y > 2147483647LL || a->n_z > 2147483647LL || a->n_y * a->n_z > 2147483647LL)
    return set_err(c, XLMIMO_EINVAL, "at most 2^31-1 elements");
  return XLMIMO_OK;
}

int check_batch(xlmimo_ctx* c, const xlmimo_batch* b, bool need_pos, int max_k = XLMIMO_MAX_USERS) {
  if (!b) return set_err(c, XLMIMO_EINVAL, "batch is NULL");
  if (b->n_drops < 0 || b->n_drops > 2147483647LL) return set_err(c, XLMIMO_EINVAL, "bad n_drops");
  if (b->n_drops == 0) return XLMIMO_OK;
  if (!b->n_users) return set_err(c, XLMIMO_EINVAL, "n_users is NULL");
  for (int64_t d = 0; d < b->n_drops; ++d) {
    if (b->n_users[d] < 1 || b->n_users[d] > max_k)
      return set_err(c, XLMIMO_EINVAL, "drop %lld: K = %d outside 1..%d", (long long)d, b->n_users[d], max_k);
    if (b->n_elems && (b->n_elems[d] < 1 || b->n_elems[d] > 2147483647LL))
      return set_err(c, XLMIMO_EINVAL, "drop %lld: N = %lld outside 1..2^31-1", (long long)d, (long long)b->n_elems[d]);
  }
  if (need_pos && !b->user_pos) return set_err(c, XLMIMO_EINVAL, "user_pos is NULL");
  return XLMIMO_OK;
}

uint64_t fnv(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ULL;
  }
  return h;
}

// Work-item length: long enough to amortise the per-item reduction, short
// enough to give the persistent grid several items per workgroup.
int64_t chunk_length(int64_t total_elems, int grid) {
  int64_t target = total_elems / (8LL * std::max(grid, 1));
  target = std::max<int64_t>(target, 2048);
  target = std::min<int64_t>(target, 65536);
  return (target + 255) / 256 * 256;  // whole rounds of every FP32 kernel (16, 128 and 256 elements)
}

uint64_t plan_key(const xlmimo_array* a, const xlmimo_batch* b, const int64_t* n_override) {
  uint64_t h = 1469598103934665603ULL;
  h = fnv(h, &a->geometry, sizeof(a->geometry));
  h = fnv(h, &a->amp_model, sizeof(a->amp_model));
  h = fnv(h, &a->n_y, sizeof(a->n_y));
  h = fnv(h, &a->n_z, sizeof(a->n_z));
  h = fnv(h, &b->n_drops, sizeof(b->n_drops));
  const int64_t flag = n_override ? *n_override : (b->n_elems ? -1 : -2);
  h = fnv(h, &flag, sizeof(flag));
  if (b->n_elems && !n_override) h = fnv(h, b->n_elems, sizeof(int64_t) * b->n_drops);
  h = fnv(h, b->n_users, sizeof(int32_t) * b->n_drops);
  return h;
}

void drop_plan_buffers(xlmimo_ctx* c, Plan& p) {
  (void)release(c, p.d_drops);
  (void)release(c, p.d_items);
  (void)release(c, p.d_v);
  (void)release(c, p.d_vmap);
  (void)release(c, p.d_vr);
  (void)release(c, p.d_mdrop);
  (void)release(c, p.d_moff);
  (void)release(c, p.d_mloc);
  p.d_mdrop = p.d_moff = p.d_mloc = nullptr;
  p.d_drops = nullptr;
  p.d_items = nullptr;
  p.d_v = nullptr;
  p.d_vmap = nullptr;
  p.d_vr = nullptr;
  if (p.vplan) {
    drop_plan_buffers(c, *p.vplan);
    delete p.vplan;
    p.vplan = nullptr;
  }
}

// Fill a plan for drops with the given N and K and upload its descriptors.
int build_plan(xlmimo_ctx* c, const xlmimo_array* a, int n, const int64_t* ne, const int32_t* kk, uint64_t h, Plan& p,
               const int32_t* cross = nullptr);

// Build (or fetch) the launch plan of a batch shape.  A cache miss uploads the
// descriptors synchronously; warm the cache before capturing a graph.
int get_plan(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, const int64_t* n_override, Plan** out) {
  const uint64_t h = plan_key(a, b, n_override);
  auto it = c->plans.find(h);
  if (it != c->plans.end()) {
    *out = &it->second;
    return XLMIMO_OK;
  }
  if (c->capturing)
    return set_err(c, XLMIMO_EINVAL, "a new batch shape needs a launch plan during graph capture: "
                   "run the same calls once before capturing them");
  if (c->plans.size() >= 64) {
    HIP_TRY(c, hipDeviceSynchronize());
    for (auto& kv : c->plans) drop_plan_buffers(c, kv.second);
    c->plans.clear();
  }
  const int n = (int)b->n_drops;
  std::vector<int64_t> ne(n);
  for (int d = 0; d < n; ++d)
    ne[d] = a->geometry == XLMIMO_UPA ? a->n_y * a->n_z
                                      : (n_override ? *n_override : (b->n_elems ? b->n_elems[d] : a->n_y));
  Plan p;
  int rc = build_plan(c, a, n, ne.data(), b->n_users, h, p);
  if (rc) {
    drop_plan_buffers(c, p);
    return rc;
  }
  if (p.k_max > XLMIMO_MAX_USERS) {
    p.ne_host = ne;
    p.k_host.assign(b->n_users, b->n_users + n);
  }
  auto ins = c->plans.emplace(h, p);
  *out = &ins.first->second;
  return XLMIMO_OK;
}

// Host layout of a batch: each drop's descriptor (its users', Gram entries', user pairs' and
// partial images' offsets) and the work items, chunk-long element ranges of every drop in
// longest-first order (stable for equal costs) for the persistent queue.  No device call.
struct HostLayout {
  std::vector<DropK> drops;
  std::vector<ItemK> items;
  int nb_max = 1, k_max = 1;
  bool has3_or_cross = false;   // a 3-block drop or a cross-only virtual drop
  int64_t total_users = 0, gram_elems = 0, n_pairs = 0, total_elems = 0, partial_doubles = 0;
};

void layout_drops(int n, const int64_t* ne_of, const int32_t* kk, const int32_t* cross, HostLayout& L) {
  L.drops.assign(n, DropK{});
  for (int d = 0; d < n; ++d) {
    DropK& dk = L.drops[d];
    const int64_t ne = ne_of[d];
    dk.n_elems = (int32_t)ne;
    dk.k = kk[d];
    dk.cross = cross ? cross[d] : 0;
    dk.nb = (dk.k + 15) / 16;
    dk.user_off = L.total_users;
    dk.gram_off = L.gram_elems;
    dk.pair_off = L.n_pairs;
    L.n_pairs += (int64_t)dk.k * (dk.k - 1) / 2;
    L.total_users += dk.k;
    L.gram_elems += (int64_t)dk.k * dk.k;
    L.total_elems += ne;
    L.nb_max = std::max(L.nb_max, dk.nb);
    L.k_max = std::max(L.k_max, dk.k);
    L.has3_or_cross = L.has3_or_cross || dk.nb == 3 || dk.cross;
  }
}

void layout_items(int64_t ch, HostLayout& L) {
  std::vector<ItemK> items;
  std::vector<int64_t> cost;
  int64_t poff = 0;
  for (size_t d = 0; d < L.drops.size(); ++d) {
    DropK& dk = L.drops[d];
    const int64_t ni = (dk.n_elems + ch - 1) / ch;
    dk.n_items = (int32_t)ni;
    dk.part_off = poff;
    poff += ni * (int64_t)partial_values(dk.nb) * 64;
    for (int64_t i = 0; i < ni; ++i) {
      ItemK itm;
      itm.drop = (int32_t)d;
      itm.chunk = (int32_t)i;
      itm.e_begin = (int32_t)(i * ch);
      itm.e_end = (int32_t)std::min<int64_t>((i + 1) * ch, dk.n_elems);
      items.push_back(itm);
      const int nb = dk.nb;
      cost.push_back((int64_t)(itm.e_end - itm.e_begin) * (nb * 8 + 3 * (nb * (nb + 1) / 2 + nb * nb)));
    }
  }
  std::vector<int> order(items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  L.items.resize(items.size());
  for (size_t i = 0; i < order.size(); ++i) L.items[i] = items[order[i]];
  L.partial_doubles = poff;
}

int build_plan(xlmimo_ctx* c, const xlmimo_array* a, int n, const int64_t* ne_of, const int32_t* kk, uint64_t h,
               Plan& p, const int32_t* cross) {
  p.n_drops = n;
  HostLayout L;
  layout_drops(n, ne_of, kk, cross, L);
  p.nb_max = L.nb_max;
  p.k_max = L.k_max;
  if (p.nb_max == 4 && !L.has3_or_cross) p.nb_max = kNbWide;
  p.total_users = L.total_users;
  p.gram_elems = L.gram_elems;
  p.n_pairs = L.n_pairs;
  p.grid_fp32 = gram_exact_grid(XLMIMO_FP32C, p.nb_max, a->geometry, a->amp_model);
  p.grid_fp64 = gram_exact_grid(XLMIMO_FP64, p.nb_max, a->geometry, a->amp_model);
  p.grid_fp32h = gram_exact_grid(XLMIMO_FP32H, p.nb_max, a->geometry, a->amp_model);
  auto tc = c->tuned_chunk.find(h);
  const int64_t ch = tc != c->tuned_chunk.end()
                         ? tc->second
                         : chunk_length(L.total_elems, std::min(std::min(p.grid_fp32, p.grid_fp64), p.grid_fp32h));
  p.chunk = ch;
  p.key = h;
  layout_items(ch, L);
  p.n_items = (int)L.items.size();
  p.partial_doubles = L.partial_doubles;
  HIP_TRY(c, hipMalloc(&p.d_drops, sizeof(DropK) * std::max(n, 1)));
  HIP_TRY(c, hipMalloc(&p.d_items, sizeof(ItemK) * std::max<size_t>(L.items.size(), 1)));
  HIP_TRY(c, hipMemcpy(p.d_drops, L.drops.data(), sizeof(DropK) * n, hipMemcpyHostToDevice));
  if (!L.items.empty())
    HIP_TRY(c, hipMemcpy(p.d_items, L.items.data(), sizeof(ItemK) * L.items.size(), hipMemcpyHostToDevice));
  return XLMIMO_OK;
}

// The virtual drops of one drop of K users.  K <= XLMIMO_MAX_USERS: one of its own (block a
// only).  A larger drop has g = ceil(K / kGroupUsers) groups (group i holds users
// [32 i, min(32 i + 32, K)), so only the last is short and it is never group a) and one
// virtual drop per group pair a < b, whose a-b block is always copied out.  The pairs
// (a, a + 1) compute their whole Gram and also give group a's own block (kVCopyA), the last
// pair also the last group's (kVCopyB); every other pair computes only the products between
// its two groups (cross).
struct GroupPair {
  int a0, ka, b0, kb, flags, cross;
};
std::vector<GroupPair> group_pairs(int K) {
  std::vector<GroupPair> out;
  if (K <= XLMIMO_MAX_USERS) {
    out.push_back({0, K, 0, 0, kVCopyA, 0});
    return out;
  }
  const int g = (K + kGroupUsers - 1) / kGroupUsers;
  auto first = [&](int i) { return std::min(K, i * kGroupUsers); };
  for (int ga = 0; ga < g; ++ga)
    for (int gb = ga + 1; gb < g; ++gb) {
      int flags = 0;
      if (gb == ga + 1) flags |= kVCopyA;
      if (ga == g - 2 && gb == g - 1) flags |= kVCopyB;
      out.push_back({first(ga), first(ga + 1) - first(ga), first(gb), first(gb + 1) - first(gb), flags, flags ? 0 : 1});
    }
  return out;
}

// Virtual drops of a batch with K > XLMIMO_MAX_USERS (every drop as group_pairs lays it out).
int build_groups(xlmimo_ctx* c, const xlmimo_array* a, Plan& p) {
  if (c->capturing)
    return set_err(c, XLMIMO_EINVAL, "a new batch shape needs a launch plan during graph capture: "
                   "run the same calls once before capturing them");
  const int n = p.n_drops;
  std::vector<VDropK> vd;
  std::vector<int64_t> vmap, vne;
  std::vector<int32_t> vk, vcross;
  int64_t uoff = 0, goff = 0, vgoff = 0;
  for (int d = 0; d < n; ++d) {
    const int K = p.k_host[d];
    auto add = [&](int a0, int ka, int b0, int kb, int flags, int cross) {
      VDropK v;
      v.gram_off = goff;
      v.vgram_off = vgoff;
      v.k = K;
      v.a0 = a0;
      v.ka = ka;
      v.b0 = b0;
      v.kb = kb;
      v.flags = flags;
      vd.push_back(v);
      for (int i = 0; i < ka; ++i) vmap.push_back(uoff + a0 + i);
      for (int i = 0; i < kb; ++i) vmap.push_back(uoff + b0 + i);
      vne.push_back(p.ne_host[d]);
      vk.push_back(ka + kb);
      vcross.push_back(cross);
      vgoff += (int64_t)(ka + kb) * (ka + kb);
    };
    for (const GroupPair& gp : group_pairs(K)) add(gp.a0, gp.ka, gp.b0, gp.kb, gp.flags, gp.cross);
    uoff += K;
    goff += (int64_t)K * K;
  }
  if (vd.size() > 2147483647ULL) return set_err(c, XLMIMO_EINVAL, "too many user-group pairs");
  Plan* vp = new Plan();
  int rc = build_plan(c, a, (int)vd.size(), vne.data(), vk.data(), p.key ^ 0x9e3779b97f4a7c15ULL, *vp,
                      vcross.data());
  if (rc) {
    drop_plan_buffers(c, *vp);
    delete vp;
    return rc;
  }
  p.vplan = vp;
  p.n_v = (int)vd.size();
  p.n_vusers = (int64_t)vmap.size();
  HIP_TRY(c, hipMalloc(&p.d_v, sizeof(VDropK) * vd.size()));
  HIP_TRY(c, hipMalloc(&p.d_vmap, sizeof(int64_t) * std::max<size_t>(vmap.size(), 1)));
  HIP_TRY(c, hipMemcpy(p.d_v, vd.data(), sizeof(VDropK) * vd.size(), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(p.d_vmap, vmap.data(), sizeof(int64_t) * vmap.size(), hipMemcpyHostToDevice));
  return XLMIMO_OK;
}

ArrayK to_kernel(const xlmimo_array* a) {
  ArrayK k;
  k.geom = a->geometry;
  k.amp = a->amp_model;
  k.n_y = (int32_t)a->n_y;
  k.n_z = (int32_t)a->n_z;
  k.spacing = a->spacing_m;
  k.lambda = a->wavelength_m;
  k.inv_lambda = 1.0 / a->wavelength_m;
  k.beta0 = a->beta0;
  return k;
}

int set_device(xlmimo_ctx* c) {
  HIP_TRY(c, hipSetDevice(c->device));
  return XLMIMO_OK;
}

// During graph capture every call must be enqueued on the capturing stream.
int stream_ok(xlmimo_ctx* c, void* stream) {
  if (c->capturing && (hipStream_t)stream != c->cap_stream)
    return set_err(c, XLMIMO_EINVAL, "during graph capture, calls must use the capturing stream");
  return XLMIMO_OK;
}

// Calls that synchronise or keep host-side state cannot be captured.
int no_capture(xlmimo_ctx* c, const char* what) {
  if (c->capturing) return set_err(c, XLMIMO_EINVAL, "%s cannot run during graph capture", what);
  return XLMIMO_OK;
}

// Persistent grid of the exact-Gram kernel: all resident workgroups, or the
// autotuned size, never more than there are work items.
int exact_grid(xlmimo_ctx* c, const Plan* p, int precision) {
  int g = precision == XLMIMO_FP64 ? p->grid_fp64 : (precision == XLMIMO_FP32H ? p->grid_fp32h : p->grid_fp32);
  auto tg = c->tuned_grid.find(p->key ^ (uint64_t)precision);
  if (tg != c->tuned_grid.end()) g = tg->second;
  return std::min(g, std::max(p->n_items, 1));
}

int run_exact(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, Plan* p, int32_t precision,
              double* gram_out, hipStream_t s);

int gram_exact_impl(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, const int64_t* n_override,
                    int32_t precision, double* gram_out, hipStream_t s) {
  Plan* p = nullptr;
  int rc = get_plan(c, a, b, n_override, &p);
  if (rc) return rc;
  if (p->k_max > XLMIMO_MAX_USERS && !p->vplan && (rc = build_groups(c, a, *p))) return rc;
  return run_exact(c, a, b, p, precision, gram_out, s);
}

// Launch the exact Gram of a plan: directly, or through its virtual drops
// (user groups or moved-user rows) and the matching scatter.
int run_exact(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, Plan* p, int32_t precision,
              double* gram_out, hipStream_t s) {
  Plan* run = p->vplan ? p->vplan : p;   // the plan whose drops the kernels see
  int rc = ensure(c, c->partials, sizeof(double) * std::max<int64_t>(run->partial_doubles, 1), s);
  if (rc) return rc;
  const double* pos = b->user_pos;
  double* out = gram_out;
  if (p->vplan) {
    if ((rc = ensure(c, c->scratch_vpos, sizeof(double) * 3 * std::max<int64_t>(p->n_vusers, 1), s))) return rc;
    if ((rc = ensure(c, c->scratch_vgram, sizeof(double) * 2 * std::max<int64_t>(run->gram_elems, 1), s))) return rc;
    HIP_TRY(c, launch_gather_users(b->user_pos, p->d_vmap, p->n_vusers, (double*)c->scratch_vpos.p, s));
    pos = (const double*)c->scratch_vpos.p;
    out = (double*)c->scratch_vgram.p;
  }
  const int grid = exact_grid(c, run, precision);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (c->timing && !c->capturing) {
    while (c->ev_pool.size() < c->ev_used + 2) {
      hipEvent_t e;
      HIP_TRY(c, hipEventCreate(&e));
      c->ev_pool.push_back(e);
    }
    ev0 = c->ev_pool[c->ev_used];
    ev1 = c->ev_pool[c->ev_used + 1];
    c->ev_used += 2;
  }
  HIP_TRY(c, launch_gram_exact(precision, run->nb_max, to_kernel(a), run->d_drops, run->n_drops, pos, run->d_items,
                               run->n_items, c->d_counter, (double*)c->partials.p, out, grid, s, ev0, ev1));
  if (p->d_vr)
    HIP_TRY(c, launch_scatter_rows(p->d_vr, p->n_vr, p->d_vmap, (const double*)c->scratch_vgram.p, gram_out, s));
  else if (p->vplan)
    HIP_TRY(c, launch_scatter_groups(p->d_v, p->n_v, (const double*)c->scratch_vgram.p, gram_out, s));
  return XLMIMO_OK;
}

// Allocation-free exact Gram (xlmimo_gram_exact_noalloc).  The launch plan is
// built on the host into a static staging buffer and copied on the stream into
// the static device array, laid out as
//   [queue counter: 256 B][DropK x n_drops][ItemK x n_items][partials]
// (each part 256-byte aligned).  No heap or device allocation is made: the
// items are sorted in place (cost descending, then drop and chunk ascending,
// the order of the context's plans).
constexpr size_t kNoallocBytes = XLMIMO_NOALLOC_SCRATCH_BYTES;
size_t align256(size_t n) { return (n + 255) / 256 * 256; }

struct NoallocState {
  std::mutex mu;
  unsigned char stage[kNoallocBytes];   // host image of the plan (DropK, then ItemK)
  hipEvent_t uploaded[64] = {};         // per device: recorded after the last plan upload
};
NoallocState& noalloc_state() {
  static NoallocState st;
  return st;
}

int gram_exact_noalloc_impl(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, int32_t precision,
                            double* gram_out, hipStream_t s) {
  if (c->device >= 64) return set_err(c, XLMIMO_EINVAL, "device %d beyond the allocation-free path's 64", c->device);
  unsigned char* dev = static_cast<unsigned char*>(static_scratch(c->device));
  if (!dev)
    return set_err(c, XLMIMO_EDEVICE, "static scratch of device %d was not set up: %s", c->device,
                   hipGetErrorString(c->scratch_init));
  const int n = (int)b->n_drops;
  int nb_max = 1;
  int64_t total_elems = 0, max_ne = 1, part_per_chunk_sum = 0;
  auto ne_of = [&](int d) -> int64_t {
    return a->geometry == XLMIMO_UPA ? a->n_y * a->n_z : (b->n_elems ? b->n_elems[d] : a->n_y);
  };
  bool has3 = false;
  for (int d = 0; d < n; ++d) {
    const int nb = (b->n_users[d] + 15) / 16;
    nb_max = std::max(nb_max, nb);
    has3 = has3 || nb == 3;
    total_elems += ne_of(d);
    max_ne = std::max(max_ne, ne_of(d));
    part_per_chunk_sum += (int64_t)partial_values(nb) * 64;
  }
  if (nb_max == 4 && !has3) nb_max = kNbWide;   // no cross-group drops here (K <= XLMIMO_MAX_USERS)
  // work-item length: the context's default for this batch, lengthened while
  // the plan and partial sums do not fit
  const int g32 = gram_exact_grid(XLMIMO_FP32C, nb_max, a->geometry, a->amp_model);
  const int g64 = gram_exact_grid(XLMIMO_FP64, nb_max, a->geometry, a->amp_model);
  const int g16 = gram_exact_grid(XLMIMO_FP32H, nb_max, a->geometry, a->amp_model);
  int64_t ch = chunk_length(total_elems, std::min(std::min(g32, g64), g16));
  const size_t drops_bytes = align256(sizeof(DropK) * (size_t)n);
  auto need = [&](int64_t chunk, int64_t* items_out) -> size_t {
    int64_t items = 0, doubles = 0;
    for (int d = 0; d < n; ++d) {
      const int64_t ni = (ne_of(d) + chunk - 1) / chunk;
      items += ni;
      doubles += ni * (int64_t)partial_values((b->n_users[d] + 15) / 16) * 64;
    }
    if (items_out) *items_out = items;
    return 256 + drops_bytes + align256(sizeof(ItemK) * (size_t)items) + sizeof(double) * (size_t)doubles;
  };
  int64_t n_items = 0;
  size_t bytes = need(ch, &n_items);
  while (bytes > kNoallocBytes && ch < max_ne) {
    ch = std::min<int64_t>(2 * ch, (max_ne + 127) / 128 * 128);
    bytes = need(ch, &n_items);
  }
  if (bytes > kNoallocBytes)
    return set_err(c, XLMIMO_EINVAL, "batch needs %zu bytes of scratch with one work item per drop; the "
                   "allocation-free exact Gram holds %zu", bytes, kNoallocBytes);
  if (n_items > 2147483647LL) return set_err(c, XLMIMO_EINVAL, "too many work items");

  NoallocState& st = noalloc_state();
  std::lock_guard<std::mutex> lk(st.mu);
  hipEvent_t& up = st.uploaded[c->device];
  if (!up) HIP_TRY(c, hipEventCreateWithFlags(&up, hipEventDisableTiming));
  else HIP_TRY(c, hipEventSynchronize(up));   // the previous upload has left the staging buffer
  DropK* drops = reinterpret_cast<DropK*>(st.stage);
  ItemK* items = reinterpret_cast<ItemK*>(st.stage + drops_bytes);
  int64_t uoff = 0, goff = 0, pairs = 0, poff = 0, it = 0;
  for (int d = 0; d < n; ++d) {
    DropK& dk = drops[d];
    dk = DropK{};
    dk.n_elems = (int32_t)ne_of(d);
    dk.k = b->n_users[d];
    dk.cross = 0;
    dk.nb = (dk.k + 15) / 16;
    dk.user_off = uoff;
    dk.gram_off = goff;
    dk.pair_off = pairs;
    pairs += (int64_t)dk.k * (dk.k - 1) / 2;
    uoff += dk.k;
    goff += (int64_t)dk.k * dk.k;
    const int64_t ni = (dk.n_elems + ch - 1) / ch;
    dk.n_items = (int32_t)ni;
    dk.part_off = poff;
    poff += ni * (int64_t)partial_values(dk.nb) * 64;
    for (int64_t i = 0; i < ni; ++i) {
      ItemK& itm = items[it++];
      itm.drop = d;
      itm.chunk = (int32_t)i;
      itm.e_begin = (int32_t)(i * ch);
      itm.e_end = (int32_t)std::min<int64_t>((i + 1) * ch, dk.n_elems);
    }
  }
  auto cost = [&](const ItemK& x) {
    const int nb = drops[x.drop].nb;
    return (int64_t)(x.e_end - x.e_begin) * (nb * 8 + 3 * (nb * (nb + 1) / 2 + nb * nb));
  };
  std::sort(items, items + n_items, [&](const ItemK& x, const ItemK& y) {
    const int64_t cx = cost(x), cy = cost(y);
    if (cx != cy) return cx > cy;
    return x.drop != y.drop ? x.drop < y.drop : x.chunk < y.chunk;
  });
  int* d_counter = reinterpret_cast<int*>(dev);
  DropK* d_drops = reinterpret_cast<DropK*>(dev + 256);
  ItemK* d_items = reinterpret_cast<ItemK*>(dev + 256 + drops_bytes);
  double* d_part = reinterpret_cast<double*>(dev + 256 + drops_bytes + align256(sizeof(ItemK) * (size_t)n_items));
  HIP_TRY(c, hipMemcpyAsync(dev + 256, st.stage, drops_bytes + sizeof(ItemK) * (size_t)n_items,
                            hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipEventRecord(up, s));
  const int grid = std::min(gram_exact_grid(precision, nb_max, a->geometry, a->amp_model), std::max((int)n_items, 1));
  HIP_TRY(c, launch_gram_exact(precision, nb_max, to_kernel(a), d_drops, n, b->user_pos, d_items, (int)n_items,
                               d_counter, d_part, gram_out, grid, s));
  return XLMIMO_OK;
}

// Row plan of a set of moved users (global indices, strictly ascending): for
// each moved user m of drop d, its partners are every other user of d except
// moved users below m (their rows already hold the entry), in runs of at most
// XLMIMO_MAX_USERS - 1; each run with m first is one virtual drop.  A user
// with no partners (K = 1, or every other user moved and below it) is a
// virtual drop of its own, for G_mm.
int get_row_plan(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, int64_t n_moved,
                 const int64_t* moved, Plan** out) {
  uint64_t h = plan_key(a, b, nullptr);
  h = fnv(h ^ 0x726f777375706474ULL, moved, sizeof(int64_t) * n_moved);
  auto it = c->row_plans.find(h);
  if (it != c->row_plans.end()) {
    *out = &it->second;
    return XLMIMO_OK;
  }
  if (c->capturing)
    return set_err(c, XLMIMO_EINVAL, "a new set of moved users needs a launch plan during graph capture: "
                   "run the same call once before capturing it");
  if (c->row_plans.size() >= 16) {   // a tracking loop with changing moved sets keeps the batch plans
    HIP_TRY(c, hipDeviceSynchronize());
    for (auto& kv : c->row_plans) drop_plan_buffers(c, kv.second);
    c->row_plans.clear();
  }
  const int n = (int)b->n_drops;
  std::vector<int64_t> uoff(n + 1, 0), goff(n + 1, 0);
  for (int d = 0; d < n; ++d) {
    uoff[d + 1] = uoff[d] + b->n_users[d];
    goff[d + 1] = goff[d] + (int64_t)b->n_users[d] * b->n_users[d];
  }
  std::vector<VRowK> vr;
  std::vector<int64_t> vmap, vne;
  std::vector<int32_t> vk, mdrop, moff, mloc;
  int64_t vgoff = 0;
  std::vector<char> is_moved;
  int cur_drop = -1;
  for (int64_t q = 0; q < n_moved; ++q) {
    const int64_t u = moved[q];
    const int d = (int)(std::upper_bound(uoff.begin(), uoff.end(), u) - uoff.begin()) - 1;
    const int K = b->n_users[d];
    if (d != cur_drop) {   // moved users of this drop, for the partner rule
      mdrop.push_back(d);
      moff.push_back((int32_t)mloc.size());
      cur_drop = d;
      is_moved.assign(K, 0);
      for (int64_t r = q; r < n_moved && moved[r] < uoff[d + 1]; ++r) is_moved[moved[r] - uoff[d]] = 1;
    }
    const int m = (int)(u - uoff[d]);
    mloc.push_back(m);
    const int64_t ne = a->geometry == XLMIMO_UPA ? a->n_y * a->n_z : (b->n_elems ? b->n_elems[d] : a->n_y);
    std::vector<int> partners;
    for (int j = 0; j < K; ++j)
      if (j != m && !(is_moved[j] && j < m)) partners.push_back(j);
    const int per = XLMIMO_MAX_USERS - 1;
    const int runs = std::max<int>(1, ((int)partners.size() + per - 1) / per);
    for (int r = 0; r < runs; ++r) {
      const int j0 = r * per, j1 = std::min<int>((int)partners.size(), j0 + per);
      VRowK v;
      v.gram_off = goff[d];
      v.vgram_off = vgoff;
      v.user_off = uoff[d];
      v.vu0 = (int64_t)vmap.size();
      v.k = K;
      v.kv = 1 + (j1 - j0);
      v.diag = r == 0;
      v.pad = 0;
      vr.push_back(v);
      vmap.push_back(u);
      for (int j = j0; j < j1; ++j) vmap.push_back(uoff[d] + partners[j]);
      vne.push_back(ne);
      vk.push_back(v.kv);
      vgoff += (int64_t)v.kv * v.kv;
    }
  }
  if (vr.size() > 2147483647ULL) return set_err(c, XLMIMO_EINVAL, "too many moved-user rows");
  Plan p;
  p.n_drops = n;
  p.key = h;
  Plan* vp = new Plan();
  p.vplan = vp;
  int rc = build_plan(c, a, (int)vr.size(), vne.data(), vk.data(), h ^ 0x9e3779b97f4a7c15ULL, *vp);
  if (!rc) {
    p.n_vr = (int)vr.size();
    p.n_vusers = (int64_t)vmap.size();
    hipError_t e = hipMalloc(&p.d_vr, sizeof(VRowK) * std::max<size_t>(vr.size(), 1));
    if (e == hipSuccess) e = hipMalloc(&p.d_vmap, sizeof(int64_t) * std::max<size_t>(vmap.size(), 1));
    if (e == hipSuccess && !vr.empty())
      e = hipMemcpy(p.d_vr, vr.data(), sizeof(VRowK) * vr.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !vmap.empty())
      e = hipMemcpy(p.d_vmap, vmap.data(), sizeof(int64_t) * vmap.size(), hipMemcpyHostToDevice);
    moff.push_back((int32_t)mloc.size());
    p.n_mdrop = (int)mdrop.size();
    if (e == hipSuccess) e = hipMalloc(&p.d_mdrop, sizeof(int32_t) * std::max<size_t>(mdrop.size(), 1));
    if (e == hipSuccess) e = hipMalloc(&p.d_moff, sizeof(int32_t) * moff.size());
    if (e == hipSuccess) e = hipMalloc(&p.d_mloc, sizeof(int32_t) * std::max<size_t>(mloc.size(), 1));
    if (e == hipSuccess && !mdrop.empty())
      e = hipMemcpy(p.d_mdrop, mdrop.data(), sizeof(int32_t) * mdrop.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p.d_moff, moff.data(), sizeof(int32_t) * moff.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !mloc.empty())
      e = hipMemcpy(p.d_mloc, mloc.data(), sizeof(int32_t) * mloc.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = set_err(c, XLMIMO_EDEVICE, "row plan upload: %s", hipGetErrorString(e));
  }
  if (rc) {
    drop_plan_buffers(c, p);
    return rc;
  }
  auto ins = c->row_plans.emplace(h, p);
  *out = &ins.first->second;
  return XLMIMO_OK;
}

int closedform_impl(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, const int64_t* n_override,
                    int32_t variant, double* gram_out, int32_t* status, hipStream_t s) {
  Plan* p = nullptr;
  int rc = get_plan(c, a, b, n_override, &p);
  if (rc) return rc;
  if ((rc = ensure(c, c->scratch_routes, sizeof(int32_t) * std::max<int64_t>(p->n_pairs, 1), s))) return rc;
  HIP_TRY(c, launch_closedform(to_kernel(a), p->d_drops, p->n_drops, variant, b->user_pos, c->d_gl, c->n_gl, nullptr,
                               gram_out, status, p->k_max, s, p->n_pairs, (int32_t*)c->scratch_routes.p));
  return XLMIMO_OK;
}

int rates_k_max(int k) { return k <= 16 ? 16 : (k <= 32 ? 32 : (k <= XLMIMO_MAX_USERS ? XLMIMO_MAX_USERS : k)); }

// Workspace of the workgroup-per-drop rate kernel: one K x K matrix per drop.
int ensure_rates_work(xlmimo_ctx* c, const Plan* p, hipStream_t s, double** work) {
  *work = nullptr;
  if (p->k_max <= XLMIMO_MAX_USERS) return XLMIMO_OK;
  int rc = ensure(c, c->scratch_work, sizeof(double) * 2 * std::max<int64_t>(p->gram_elems, 1), s);
  if (rc) return rc;
  *work = (double*)c->scratch_work.p;
  return XLMIMO_OK;
}

}  // namespace

struct xlmimo_mlp {
  xlmimo_ctx* ctx = nullptr;
  int width = 0, depth = 0, n_layers = 0;
  std::vector<int> in_dim, out_dim;
  std::vector<int64_t> w_off, b_off;
  int64_t n_params = 0;
  float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  __bf16* wbf = nullptr;
  __bf16* wbf_t = nullptr;    // per layer, the weights transposed ([in][out] BF16; input gradients)
  xl::SplitLayers dims{};     // layer table (start = weight offset, in_dim) for the per-parameter kernels
  int64_t* d_offs = nullptr;  // per layer: weight offset, bias offset (fused inference)
  int64_t t = 0;
  DevBuf act, partial, split, loss_scratch;
  // fallback gate by antenna count (xlmimo_mlp_set_gate)
  std::vector<int64_t> gate_n;
  std::vector<double> gate_thr;
};

namespace {

constexpr int kFeatPitch = 8;   // features per pair (6 used)
constexpr int kAuxPitch = 8;    // phasors (6), closed-form scale, pad
constexpr int kOut = 7;

// Activation layout for a batch of n pairs: per hidden layer, the GELU output
// (bf16, next layer's input) and the pre-activation (fp32); the network output;
// two bf16 gradient buffers and the output gradient.
struct Acts {
  std::vector<__bf16*> x;   // x[l] = input of layer l for l >= 1
  std::vector<float*> z;    // z[l] = pre-activation of hidden layer l
  std::vector<__bf16*> dz;  // dz[l] = gradient at the pre-activation of hidden layer l (training)
  float* out = nullptr;
  __bf16 *da = nullptr, *db = nullptr, *dout = nullptr;
};

int mlp_acts(xlmimo_ctx* c, xlmimo_mlp* M, int64_t n, bool train, Acts& a, hipStream_t s) {
  const int H = M->width, L = M->n_layers;
  size_t bytes = 0;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t xb = al(sizeof(__bf16) * n * H), zb = al(sizeof(float) * n * H);
  const size_t ob = al(sizeof(float) * n * kOut), dob = al(sizeof(__bf16) * n * kDoutPitch);
  const int n_dz = std::max(2, L - 1);
  bytes = (train ? (L - 1) * (xb + zb) + n_dz * xb + dob : 2 * xb) + ob;
  int rc = ensure(c, M->act, bytes, s);
  if (rc) return rc;
  char* p = (char*)M->act.p;
  a.x.assign(L, nullptr);
  a.z.assign(L, nullptr);
  if (train) {
    for (int l = 1; l < L; ++l) { a.x[l] = (__bf16*)p; p += xb; }
    for (int l = 0; l < L - 1; ++l) { a.z[l] = (float*)p; p += zb; }
    a.dz.assign(n_dz, nullptr);
    for (int l = 0; l < n_dz; ++l) { a.dz[l] = (__bf16*)p; p += xb; }
    a.da = a.dz[0];
    a.db = a.dz[1];
    a.dout = (__bf16*)p; p += dob;
  } else {
    // inference ping-pongs two activation buffers
    __bf16* x0 = (__bf16*)p; p += xb;
    __bf16* x1 = (__bf16*)p; p += xb;
    for (int l = 1; l < L; ++l) a.x[l] = (l & 1) ? x0 : x1;
  }
  a.out = (float*)p;
  return XLMIMO_OK;
}

int mlp_forward(xlmimo_ctx* c, xlmimo_mlp* M, int64_t n, const __bf16* feat, const Acts& a, bool keep_z,
                hipStream_t s) {
  if (keep_z && (M->width == 64 || M->width == 128 || M->width == 256)) {
    // one fused pass through every layer (activations in LDS), storing what the backward reads
    FwdKeep keep{};
    for (int l = 0; l + 1 < M->n_layers; ++l) {
      keep.z[l] = a.z[l];
      keep.x[l + 1] = a.x[l + 1];
    }
    HIP_TRY(c, launch_mlp_fused_train_forward(M->width, M->depth, n, feat, M->wbf, M->master, M->d_offs, keep, a.out, s));
    return XLMIMO_OK;
  }
  for (int l = 0; l < M->n_layers; ++l) {
    GemmArgs g{};
    g.M = (int)n;
    g.N = M->out_dim[l];
    g.K = M->in_dim[l];
    g.A = l == 0 ? feat : a.x[l];
    g.a_m = l == 0 ? kFeatPitch : M->width;
    g.a_k = 1;
    g.B = M->wbf + M->w_off[l];
    g.b_k = 1;
    g.b_n = M->in_dim[l];
    g.bias = M->master + M->b_off[l];
    if (l < M->n_layers - 1) {
      g.Z = keep_z ? a.z[l] : nullptr;
      g.out_bf = a.x[l + 1];
      g.ldo = M->width;
      HIP_TRY(c, launch_gemm(EPI_FWD_HIDDEN, g, s));
    } else {
      g.out_f = a.out;
      g.ldo = kOut;
      HIP_TRY(c, launch_gemm(EPI_FWD_OUT, g, s));
    }
  }
  return XLMIMO_OK;
}

// Split of the batch dimension for the weight-gradient GEMMs (dZ^T X reduces over pairs).
constexpr int kGradSplits = 32;
constexpr int64_t kGradSplitK = 512;   // pairs per split of the weight-gradient GEMMs

// Inference outputs [n][XLMIMO_MLP_OUT] into `out`: fused single-kernel path for
// widths 64/128/256, layer-by-layer GEMMs otherwise.
int mlp_infer(xlmimo_ctx* c, xlmimo_mlp* M, int64_t n, const __bf16* feat, float* out, hipStream_t s) {
  if (M->width == 64 || M->width == 128 || M->width == 256) {
    HIP_TRY(c, launch_mlp_fused_forward(M->width, M->depth, n, feat, M->wbf, M->master, M->d_offs, out, s));
    return XLMIMO_OK;
  }
  const int64_t chunk = 1 << 20;
  for (int64_t off = 0; off < n; off += chunk) {
    const int64_t m = std::min(chunk, n - off);
    Acts acts;
    int rc = mlp_acts(c, M, m, false, acts, s);
    if (rc) return rc;
    if ((rc = mlp_forward(c, M, m, feat + off * kFeatPitch, acts, false, s))) return rc;
    HIP_TRY(c, hipMemcpyAsync(out + off * kOut, acts.out, sizeof(float) * m * kOut, hipMemcpyDeviceToDevice, s));
  }
  return XLMIMO_OK;
}

// The weight-gradient GEMMs' split-K slices of all layers stay unreduced (to be summed by the
// Adam kernel, or by one reduction over all layers) when they fit this budget; larger networks
// reduce each layer's slices right after its GEMM.
constexpr size_t kKeepSliceBytes = size_t(256) << 20;

int grad_splits(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(kGradSplits, n / kGradSplitK)); }

bool keep_slices(const xlmimo_mlp* M, int64_t n) {
  size_t all = 0;
  for (int l = 0; l < M->n_layers; ++l) all += (size_t)grad_splits(n) * M->out_dim[l] * (M->in_dim[l] + 1);
  return all * sizeof(float) <= kKeepSliceBytes;
}

// Backward pass. With keep, the weight gradients are left as split-K slices described by *L
// (L->n = 0 otherwise: M->grad holds the reduced gradients).
int mlp_backward(xlmimo_ctx* c, xlmimo_mlp* M, int64_t n, const __bf16* feat, const Acts& a, bool keep,
                 SplitLayers* L, hipStream_t s) {
  const int splits_req = grad_splits(n);
  size_t need = 0;
  for (int l = 0; l < M->n_layers; ++l) {
    const size_t nl = (size_t)splits_req * M->out_dim[l] * (M->in_dim[l] + 1);
    need = keep ? need + nl : std::max(need, nl);
  }
  int rc = ensure(c, M->split, sizeof(float) * need, s);
  if (rc) return rc;
  float* part = (float*)M->split.p;
  L->n = keep ? M->n_layers : 0;
  if (keep) {
    // the input gradients layer by layer (each hidden layer's own buffer), then every layer's
    // weight and bias gradients in one grouped launch
    const int NL = M->n_layers;
    std::vector<const __bf16*> dzs(NL);
    std::vector<int64_t> ldzs(NL);
    dzs[NL - 1] = a.dout;
    ldzs[NL - 1] = kDoutPitch;
    const bool fused_dx = M->width == 64 || M->width == 128 || M->width == 256;
    if (fused_dx) {
      // the whole chain in one pass (gradients in LDS), storing every hidden layer's dZ
      BwdKeep bk{};
      for (int l = 0; l + 1 < NL; ++l) {
        bk.z[l] = a.z[l];
        bk.dz[l] = a.dz[l];
        dzs[l] = a.dz[l];
        ldzs[l] = M->in_dim[l + 1];
      }
      HIP_TRY(c, launch_mlp_fused_train_backward(M->width, M->depth, n, a.dout, M->wbf_t, M->d_offs, bk, s));
    }
    for (int l = NL - 1; l >= 1 && !fused_dx; --l) {
      GemmArgs gx{};
      gx.M = (int)n;
      gx.N = M->in_dim[l];
      gx.K = M->out_dim[l];
      gx.A = dzs[l];
      gx.a_m = ldzs[l];
      gx.a_k = 1;
      gx.B = M->wbf_t + M->w_off[l];   // B(k = output, n = input) with k contiguous
      gx.b_k = 1;
      gx.b_n = M->out_dim[l];
      gx.Z = a.z[l - 1];
      gx.out_bf = a.dz[l - 1];
      gx.ldo = M->in_dim[l];
      HIP_TRY(c, launch_gemm(EPI_BWD_DX, gx, s));
      dzs[l - 1] = a.dz[l - 1];
      ldzs[l - 1] = M->in_dim[l];
    }
    std::vector<GemmArgs> gs(NL);
    std::vector<int> req(NL, splits_req), slices(NL, 0);
    std::vector<float*> parts(NL);
    int64_t off = 0;
    for (int l = 0; l < NL; ++l) {
      const int in = M->in_dim[l], o = M->out_dim[l];
      GemmArgs& gw = gs[l];
      gw = GemmArgs{};
      gw.M = o;
      gw.N = in;
      gw.K = (int)n;
      gw.A = dzs[l];
      gw.a_m = 1;
      gw.a_k = ldzs[l];
      gw.B = l == 0 ? feat : a.x[l];
      gw.b_k = l == 0 ? kFeatPitch : M->width;
      gw.b_n = 1;
      gw.ldo = in;
      gw.row_sums = 1;   // the bias gradient sum_pairs dZ follows W's gradient (b_off = w_off + o in)
      parts[l] = part + off;
      L->part_off[l] = off;
      off += (int64_t)splits_req * o * (in + 1);
    }
    HIP_TRY(c, launch_gemm_grouped_partials(gs.data(), req.data(), parts.data(), NL, slices.data(), s));
    for (int l = 0; l < NL; ++l) {
      L->splits[l] = slices[l];
      L->in_dim[l] = M->in_dim[l];
      L->start[l] = M->w_off[l];
    }
    L->start[NL] = M->n_params;
    return XLMIMO_OK;
  }
  const __bf16* dz = a.dout;
  int64_t ldz = kDoutPitch;
  __bf16* bufs[2] = {a.da, a.db};
  int flip = 0;
  for (int l = M->n_layers - 1; l >= 0; --l) {
    const int in = M->in_dim[l], o = M->out_dim[l];
    const __bf16* x = l == 0 ? feat : a.x[l];
    const int64_t ldx = l == 0 ? kFeatPitch : M->width;
    GemmArgs gw{};
    gw.M = o;
    gw.N = in;
    gw.K = (int)n;
    gw.A = dz;
    gw.a_m = 1;
    gw.a_k = ldz;
    gw.B = x;
    gw.b_k = ldx;
    gw.b_n = 1;
    gw.ldo = in;
    gw.row_sums = 1;   // the bias gradient sum_pairs dZ follows W's gradient (b_off = w_off + o in)
    HIP_TRY(c, launch_gemm_splitk(gw, splits_req, part, M->grad + M->w_off[l], s));
    if (l > 0) {
      GemmArgs gx{};
      gx.M = (int)n;
      gx.N = in;
      gx.K = o;
      gx.A = dz;
      gx.a_m = ldz;
      gx.a_k = 1;
      gx.B = M->wbf + M->w_off[l];
      gx.b_k = in;
      gx.b_n = 1;
      gx.Z = a.z[l - 1];
      gx.out_bf = bufs[flip];
      gx.ldo = in;
      HIP_TRY(c, launch_gemm(EPI_BWD_DX, gx, s));
      dz = bufs[flip];
      ldz = in;
      flip ^= 1;
    }
  }
  return XLMIMO_OK;
}

// Loss and gradients of one batch.  With fused != nullptr and slices that fit, the gradients
// and the loss are left for launch_adam_layers (*fused describes the slices; the loss head's
// block partials are in M->partial); otherwise (fused->n = 0) M->grad and *loss_out are final.
int mlp_loss_grad_impl(xlmimo_ctx* c, xlmimo_mlp* M, int64_t n, const __bf16* feat, const float* aux,
                       const float* target, double* loss_out, hipStream_t s, SplitLayers* fused = nullptr) {
  Acts a;
  int rc = mlp_acts(c, M, n, true, a, s);
  if (rc) return rc;
  if ((rc = ensure(c, M->partial, sizeof(double) * kMlpHeadBlocks, s))) return rc;
  if ((rc = mlp_forward(c, M, n, feat, a, true, s))) return rc;
  const bool keep = keep_slices(M, n);
  const bool fuse = fused != nullptr && keep;
  HIP_TRY(c, launch_mlp_head(n, a.out, aux, target, a.dout, (double*)M->partial.p, fuse ? nullptr : loss_out, s));
  SplitLayers L{};
  if ((rc = mlp_backward(c, M, n, feat, a, keep, &L, s))) return rc;
  if (keep && !fuse) HIP_TRY(c, launch_reduce_layers(L, (const float*)M->split.p, M->grad, s));
  if (fused != nullptr) {
    *fused = L;
    if (!fuse) fused->n = 0;
  }
  return XLMIMO_OK;
}

// One Adam step after mlp_loss_grad_impl(..., &L): fused with the gradient reduction and the
// loss sum when L.n > 0.
int mlp_adam(xlmimo_ctx* c, xlmimo_mlp* M, const SplitLayers& L, int64_t n, float lr, double* loss_out,
             hipStream_t s) {
  M->t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.0f - std::pow(b1, (float)M->t), bc2 = 1.0f - std::pow(b2, (float)M->t);
  if (L.n > 0) {
    HIP_TRY(c, launch_adam_layers(L, (const float*)M->split.p, nullptr, M->n_params, M->master, M->m, M->v, lr, b1, b2,
                                  1e-8f, bc1, bc2, M->wbf, M->wbf_t, (const double*)M->partial.p, kMlpHeadBlocks, n,
                                  loss_out, s));
  } else {
    HIP_TRY(c, launch_adam_layers(M->dims, nullptr, M->grad, M->n_params, M->master, M->m, M->v, lr, b1, b2, 1e-8f,
                                  bc1, bc2, M->wbf, M->wbf_t, nullptr, 0, n, nullptr, s));
  }
  return XLMIMO_OK;
}

int check_mlp_args(xlmimo_ctx* c, const xlmimo_mlp* M, int64_t n, const void* feat, const void* aux) {
  if (!M || M->ctx != c) return set_err(c, XLMIMO_EINVAL, "mlp is NULL or belongs to another context");
  if (n < 0 || n > (1LL << 31) - 1) return set_err(c, XLMIMO_EINVAL, "bad pair count");
  if (n > 0 && (!feat || !aux)) return set_err(c, XLMIMO_EINVAL, "features and aux are required");
  return XLMIMO_OK;
}

int closedform_mlp_impl(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, const int64_t* n_override,
                        int32_t variant, xlmimo_mlp* M, double log_var_max, double* gram_out, int32_t* status,
                        hipStream_t s, int32_t** flags_out = nullptr);


}  // namespace


namespace {

// Closed form, then the learned residual for every pair; drops whose predicted
// log-variance exceeds log_var_max anywhere are recomputed with the exact FP32H
// Gram (same launch plan, drop mask) and flagged XLMIMO_ST_FELL_BACK.
int closedform_mlp_impl(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, const int64_t* n_override,
                        int32_t variant, xlmimo_mlp* M, double log_var_max, double* gram_out, int32_t* status,
                        hipStream_t s, int32_t** flags_out) {
  Plan* p = nullptr;
  int rc = get_plan(c, a, b, n_override, &p);
  if (rc) return rc;
  if ((rc = ensure(c, c->scratch_routes, sizeof(int32_t) * std::max<int64_t>(p->n_pairs, 1), s))) return rc;
  GateK gate{};
  gate.cap = (float)log_var_max;
  gate.n_bins = (int32_t)M->gate_n.size();
  for (int i = 0; i < gate.n_bins; ++i) {
    gate.n_upper[i] = M->gate_n[i];
    gate.thr[i] = (float)M->gate_thr[i];
  }
  // a batch whose every drop falls in a bin (or under a cap) of -inf falls back whole: the
  // network and its inputs are skipped
  bool all_fall_back = !(gate.cap > -INFINITY);
  if (!all_fall_back && gate.n_bins > 0) {
    all_fall_back = true;
    for (int d = 0; d < (int)b->n_drops && all_fall_back; ++d) {
      const int64_t ne = n_override ? *n_override : (b->n_elems ? b->n_elems[d] : a->n_y);
      float thr = gate.cap;
      for (int i = 0; i < gate.n_bins; ++i)
        if (ne <= gate.n_upper[i]) {
          thr = std::min(thr, gate.thr[i]);
          break;
        }
      all_fall_back = !(thr > -INFINITY);
    }
  }
  const int64_t np = p->n_pairs;
  const size_t fb = (sizeof(__bf16) * kFeatPitch * np + 255) / 256 * 256;
  const size_t ab = (sizeof(float) * kAuxPitch * np + 255) / 256 * 256;
  const size_t pb = (sizeof(int32_t) * 2 * np + 255) / 256 * 256;
  const size_t flb = (sizeof(int32_t) * p->n_drops + 255) / 256 * 256;
  const size_t ob = (sizeof(float) * kOut * np + 255) / 256 * 256;
  const size_t ib = (sizeof(ItemK) * std::max(p->n_items, 1) + 256 + 255) / 256 * 256;   // selected items + count
  if ((rc = ensure(c, c->scratch_pairs, fb + ab + pb + flb + ob + ib, s))) return rc;
  char* base = (char*)c->scratch_pairs.p;
  __bf16* feat = (__bf16*)base;
  float* aux = (float*)(base + fb);
  int32_t* pmap = (int32_t*)(base + fb + ab);
  int32_t* flags = (int32_t*)(base + fb + ab + pb);
  float* net_out = (float*)(base + fb + ab + pb + flb);
  ItemK* items_sel = (ItemK*)(base + fb + ab + pb + flb + ob);
  int* n_sel = (int*)(base + fb + ab + pb + flb + ob + ib - 256);
  if (all_fall_back) {
    // the exact Gram overwrites every drop; the status words still get the closed form's bits
    if (status)
      HIP_TRY(c, launch_closedform(to_kernel(a), p->d_drops, p->n_drops, variant, b->user_pos, c->d_gl, c->n_gl,
                                   nullptr, gram_out, status, p->k_max, s, p->n_pairs,
                                   (int32_t*)c->scratch_routes.p));
    HIP_TRY(c, launch_fill_i32(flags, p->n_drops, 1, s));
  } else {
    HIP_TRY(c, launch_closedform(to_kernel(a), p->d_drops, p->n_drops, variant, b->user_pos, c->d_gl, c->n_gl, nullptr,
                                 gram_out, status, p->k_max, s, p->n_pairs, (int32_t*)c->scratch_routes.p));
    HIP_TRY(c, launch_fill_i32(flags, p->n_drops, 0, s));
    HIP_TRY(c, launch_pair_inputs(to_kernel(a), p->d_drops, p->n_drops, b->user_pos, gram_out, nullptr, feat, aux,
                                  nullptr, pmap, s));
    if ((rc = mlp_infer(c, M, np, feat, net_out, s))) return rc;
    HIP_TRY(c, launch_mlp_apply(np, net_out, aux, pmap, p->d_drops, gram_out, flags, gate, s));
  }
  if ((rc = ensure(c, c->partials, sizeof(double) * std::max<int64_t>(p->partial_doubles, 1), s))) return rc;
  const int grid = exact_grid(c, p, XLMIMO_FP32H);
  HIP_TRY(c, launch_gram_exact(XLMIMO_FP32H, p->nb_max, to_kernel(a), p->d_drops, p->n_drops, b->user_pos, p->d_items,
                               p->n_items, c->d_counter, (double*)c->partials.p, gram_out, grid, s, nullptr, nullptr,
                               flags, items_sel, n_sel));
  if (status) HIP_TRY(c, launch_or_flags(status, flags, p->n_drops, XLMIMO_ST_FELL_BACK, s));
  if (flags_out) *flags_out = flags;
  return XLMIMO_OK;
}

}  // namespace

extern "C" {

int xlmimo_mlp_create(xlmimo_ctx* c, int32_t width, int32_t depth, xlmimo_mlp** out) {
  if (!c || !out) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = no_capture(c, "xlmimo_mlp_create")) return rc0;
  *out = nullptr;
  if (width < 16 || width > 4096 || width % 16) return set_err(c, XLMIMO_EINVAL, "width must be a multiple of 16 in 16..4096");
  if (depth < 1 || depth > 16) return set_err(c, XLMIMO_EINVAL, "depth must lie in 1..16");
  int rc = set_device(c);
  if (rc) return rc;
  xlmimo_mlp* M = new xlmimo_mlp();
  M->ctx = c;
  M->width = width;
  M->depth = depth;
  M->n_layers = depth + 1;
  int64_t off = 0;
  for (int l = 0; l < M->n_layers; ++l) {
    const int in = l == 0 ? XLMIMO_MLP_IN : width, o = l == depth ? XLMIMO_MLP_OUT : width;
    M->in_dim.push_back(in);
    M->out_dim.push_back(o);
    M->w_off.push_back(off);
    off += (int64_t)in * o;
    M->b_off.push_back(off);
    off += o;
  }
  M->n_params = off;
  M->dims.n = M->n_layers;
  for (int l = 0; l < M->n_layers; ++l) {
    M->dims.start[l] = M->w_off[l];
    M->dims.in_dim[l] = M->in_dim[l];
  }
  M->dims.start[M->n_layers] = off;
  const size_t fb = sizeof(float) * off;
  if (hipMalloc(&M->master, fb) || hipMalloc(&M->m, fb) || hipMalloc(&M->v, fb) || hipMalloc(&M->grad, fb) ||
      hipMalloc(&M->wbf, sizeof(__bf16) * off) || hipMalloc(&M->wbf_t, sizeof(__bf16) * off) ||
      hipMemset(M->master, 0, fb) || hipMemset(M->m, 0, fb) || hipMemset(M->v, 0, fb) ||
      hipMemset(M->grad, 0, fb) || hipMemset(M->wbf, 0, sizeof(__bf16) * off) ||
      hipMemset(M->wbf_t, 0, sizeof(__bf16) * off)) {
    (void)hipGetLastError();
    (void)hipFree(M->master); (void)hipFree(M->m); (void)hipFree(M->v); (void)hipFree(M->grad); (void)hipFree(M->wbf);
    (void)hipFree(M->wbf_t);
    delete M;
    return set_err(c, XLMIMO_ENOMEM, "MLP parameter allocation failed");
  }
  std::vector<int64_t> offs;
  for (int l = 0; l < M->n_layers; ++l) {
    offs.push_back(M->w_off[l]);
    offs.push_back(M->b_off[l]);
  }
  if (hipMalloc(&M->d_offs, sizeof(int64_t) * offs.size()) ||
      hipMemcpy(M->d_offs, offs.data(), sizeof(int64_t) * offs.size(), hipMemcpyHostToDevice)) {
    (void)hipGetLastError();
    (void)hipFree(M->master); (void)hipFree(M->m); (void)hipFree(M->v); (void)hipFree(M->grad); (void)hipFree(M->wbf);
    (void)hipFree(M->wbf_t); (void)hipFree(M->d_offs);
    delete M;
    return set_err(c, XLMIMO_ENOMEM, "MLP offset table allocation failed");
  }
  *out = M;
  return XLMIMO_OK;
}

int xlmimo_mlp_destroy(xlmimo_mlp* M) {
  if (!M) return XLMIMO_OK;
  xlmimo_ctx* c = M->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->capturing || c->graphs > 0)
    return set_err(c, XLMIMO_EINVAL, "destroy the context's graphs before its networks");
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(M->master); (void)hipFree(M->m); (void)hipFree(M->v); (void)hipFree(M->grad); (void)hipFree(M->wbf);
  (void)hipFree(M->wbf_t);
  if (M->act.p) (void)hipFree(M->act.p);
  if (M->partial.p) (void)hipFree(M->partial.p);
  if (M->split.p) (void)hipFree(M->split.p);
  if (M->loss_scratch.p) (void)hipFree(M->loss_scratch.p);
  (void)hipFree(M->d_offs);
  delete M;
  return XLMIMO_OK;
}

int64_t xlmimo_mlp_param_count(const xlmimo_mlp* M) { return M ? M->n_params : -1; }

int xlmimo_mlp_set_params(xlmimo_mlp* M, const float* host) {
  if (!M || !host) return XLMIMO_EINVAL;
  xlmimo_ctx* c = M->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = no_capture(c, "xlmimo_mlp_set_params")) return rc0;
  int rc = set_device(c);
  if (rc) return rc;
  const size_t fb = sizeof(float) * M->n_params;
  HIP_TRY(c, hipDeviceSynchronize());
  HIP_TRY(c, hipMemcpy(M->master, host, fb, hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemset(M->m, 0, fb));
  HIP_TRY(c, hipMemset(M->v, 0, fb));
  HIP_TRY(c, launch_to_bf16(M->n_params, M->master, M->wbf, nullptr));
  HIP_TRY(c, launch_weights_t(M->dims, M->master, M->wbf_t, nullptr));
  HIP_TRY(c, hipDeviceSynchronize());
  M->t = 0;
  return XLMIMO_OK;
}

int xlmimo_mlp_get_params(xlmimo_mlp* M, float* host) {
  if (!M || !host) return XLMIMO_EINVAL;
  xlmimo_ctx* c = M->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = no_capture(c, "xlmimo_mlp_get_params")) return rc0;
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, hipDeviceSynchronize());
  HIP_TRY(c, hipMemcpy(host, M->master, sizeof(float) * M->n_params, hipMemcpyDeviceToHost));
  return XLMIMO_OK;
}

int xlmimo_mlp_set_gate(xlmimo_mlp* M, int32_t n_bins, const int64_t* n_upper, const double* log_var_max) {
  if (!M) return XLMIMO_EINVAL;
  xlmimo_ctx* c = M->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  if (n_bins < 0 || n_bins > kGateBins)
    return set_err(c, XLMIMO_EINVAL, "gate bins %d outside 0..%d", n_bins, kGateBins);
  if (n_bins > 0 && (!n_upper || !log_var_max)) return set_err(c, XLMIMO_EINVAL, "gate arrays are NULL");
  for (int i = 0; i < n_bins; ++i) {
    if (n_upper[i] < 1 || (i > 0 && n_upper[i] <= n_upper[i - 1]))
      return set_err(c, XLMIMO_EINVAL, "gate bounds must be >= 1 and strictly ascending");
    if (std::isnan(log_var_max[i])) return set_err(c, XLMIMO_EINVAL, "gate threshold %d is NaN", i);
  }
  M->gate_n.assign(n_upper, n_upper + n_bins);
  M->gate_thr.assign(log_var_max, log_var_max + n_bins);
  return XLMIMO_OK;
}

int64_t xlmimo_pair_count(const xlmimo_batch* b) {
  if (!b || b->n_drops < 0 || (b->n_drops > 0 && !b->n_users)) return -1;
  int64_t n = 0;
  for (int64_t d = 0; d < b->n_drops; ++d) n += (int64_t)b->n_users[d] * (b->n_users[d] - 1) / 2;
  return n;
}

int xlmimo_mlp_pair_inputs(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, const double* gram_cf,
                           const double* gram_exact, void* features, float* aux, float* target, int32_t* pair_map,
                           void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = stream_ok(c, stream)) return rc0;
  int rc = check_array(c, a);
  if (!rc) rc = check_batch(c, b, true);
  if (rc) return rc;
  if (a->geometry != XLMIMO_ULA) return set_err(c, XLMIMO_EINVAL, "the learned correction is defined for a ULA");
  if (b->n_drops == 0) return XLMIMO_OK;
  if (!gram_cf || !features || !aux || !pair_map) return set_err(c, XLMIMO_EINVAL, "gram_cf, features, aux and pair_map are required");
  if (target && !gram_exact) return set_err(c, XLMIMO_EINVAL, "targets need gram_exact");
  if ((rc = set_device(c))) return rc;
  Plan* p = nullptr;
  if ((rc = get_plan(c, a, b, nullptr, &p))) return rc;
  HIP_TRY(c, launch_pair_inputs(to_kernel(a), p->d_drops, p->n_drops, b->user_pos, gram_cf, gram_exact,
                                (__bf16*)features, aux, target, pair_map, (hipStream_t)stream));
  return XLMIMO_OK;
}

int xlmimo_mlp_loss_grad(xlmimo_ctx* c, xlmimo_mlp* M, int64_t n, const void* features, const float* aux,
                         const float* target, float* grad_out, double* loss_out, void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = stream_ok(c, stream)) return rc0;
  int rc = check_mlp_args(c, M, n, features, aux);
  if (rc) return rc;
  if (n < 1 || !target || !loss_out) return set_err(c, XLMIMO_EINVAL, "need n >= 1, targets and loss_out");
  if ((rc = set_device(c))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if ((rc = mlp_loss_grad_impl(c, M, n, (const __bf16*)features, aux, target, loss_out, s))) return rc;
  if (grad_out) HIP_TRY(c, hipMemcpyAsync(grad_out, M->grad, sizeof(float) * M->n_params, hipMemcpyDeviceToDevice, s));
  return XLMIMO_OK;
}

int xlmimo_mlp_train_step(xlmimo_ctx* c, xlmimo_mlp* M, int64_t n, const void* features, const float* aux,
                          const float* target, float lr, double* loss_out, void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = no_capture(c, "xlmimo_mlp_train_step (its Adam step count lives on the host)")) return rc0;
  int rc = check_mlp_args(c, M, n, features, aux);
  if (rc) return rc;
  if (n < 1 || !target || !loss_out) return set_err(c, XLMIMO_EINVAL, "need n >= 1, targets and loss_out");
  if (!(lr >= 0.0f) || !std::isfinite(lr)) return set_err(c, XLMIMO_EINVAL, "bad learning rate");
  if ((rc = set_device(c))) return rc;
  hipStream_t s = (hipStream_t)stream;
  SplitLayers L{};
  if ((rc = mlp_loss_grad_impl(c, M, n, (const __bf16*)features, aux, target, loss_out, s, &L))) return rc;
  return mlp_adam(c, M, L, n, lr, loss_out, s);
}

int xlmimo_mlp_train(xlmimo_ctx* c, xlmimo_mlp* M, int64_t n, const void* features, const float* aux,
                     const float* target, int64_t batch, int64_t n_steps, const float* lr, double* loss_out,
                     void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = no_capture(c, "xlmimo_mlp_train (its Adam step count lives on the host)")) return rc0;
  int rc = check_mlp_args(c, M, n, features, aux);
  if (rc) return rc;
  if (!target || !lr) return set_err(c, XLMIMO_EINVAL, "targets and learning rates are needed");
  if (batch < 1 || batch > n || n_steps < 0) return set_err(c, XLMIMO_EINVAL, "need 1 <= batch <= n and n_steps >= 0");
  for (int64_t i = 0; i < n_steps; ++i)
    if (!(lr[i] >= 0.0f) || !std::isfinite(lr[i])) return set_err(c, XLMIMO_EINVAL, "bad learning rate at step %lld",
                                                                (long long)i);
  if ((rc = set_device(c))) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (!loss_out && (rc = ensure(c, M->loss_scratch, sizeof(double), s))) return rc;
  const int64_t n_batches = n / batch;
  const __bf16* feat = (const __bf16*)features;
  for (int64_t i = 0; i < n_steps; ++i) {
    const int64_t off = (i % n_batches) * batch;
    double* lo = loss_out ? loss_out + i : (double*)M->loss_scratch.p;
    SplitLayers L{};
    if ((rc = mlp_loss_grad_impl(c, M, batch, feat + off * kFeatPitch, aux + off * kAuxPitch, target + off * 2, lo, s,
                                 &L)))
      return rc;
    if ((rc = mlp_adam(c, M, L, batch, lr[i], lo, s))) return rc;
  }
  return XLMIMO_OK;
}

int xlmimo_mlp_forward(xlmimo_ctx* c, xlmimo_mlp* M, int64_t n, const void* features, float* out, void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = stream_ok(c, stream)) return rc0;
  int rc = check_mlp_args(c, M, n, features, (const void*)1);
  if (rc) return rc;
  if (n == 0) return XLMIMO_OK;
  if (!out) return set_err(c, XLMIMO_EINVAL, "out is NULL");
  if ((rc = set_device(c))) return rc;
  return mlp_infer(c, M, n, (const __bf16*)features, out, (hipStream_t)stream);
}

int xlmimo_gram_closedform_mlp(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, int32_t variant,
                               xlmimo_mlp* M, double log_var_max, double* gram_out, int32_t* status_out,
                               void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = stream_ok(c, stream)) return rc0;
  int rc = check_array(c, a);
  if (!rc) rc = check_batch(c, b, true);
  if (rc) return rc;
  if (a->geometry != XLMIMO_ULA) return set_err(c, XLMIMO_EINVAL, "the learned correction is defined for a ULA");
  if (variant < XLMIMO_CF_PAPER || variant > XLMIMO_CF_GATED_QUAD) return set_err(c, XLMIMO_EINVAL, "bad variant %d", variant);
  if (variant >= XLMIMO_CF_UNIFORM && a->geometry != XLMIMO_ULA)
    return set_err(c, XLMIMO_EINVAL, "closed-form variant %d is defined for a ULA", variant);
  if (!M || M->ctx != c) return set_err(c, XLMIMO_EINVAL, "mlp is NULL or belongs to another context");
  if (std::isnan(log_var_max)) return set_err(c, XLMIMO_EINVAL, "log_var_max is NaN");
  if (b->n_drops == 0) return XLMIMO_OK;
  if (!gram_out) return set_err(c, XLMIMO_EINVAL, "gram_out is NULL");
  if ((rc = set_device(c))) return rc;
  return closedform_mlp_impl(c, a, b, nullptr, variant, M, log_var_max, gram_out, status_out, (hipStream_t)stream);
}

}  // extern "C"

extern "C" {

const char* xlmimo_version(void) { return "xlmimo 0.1 (gfx950)"; }

int xlmimo_ctx_create(xlmimo_ctx** out, int device) {
  if (!out) return XLMIMO_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return XLMIMO_EDEVICE;
  }
  xlmimo_ctx* c = new xlmimo_ctx();
  c->device = device;
  if (hipSetDevice(device) != hipSuccess || hipMalloc(&c->d_counter, sizeof(int)) != hipSuccess) {
    delete c;
    return XLMIMO_EDEVICE;
  }
  // the allocation-free exact Gram's static array: its address on this device
  // (a failure is reported by xlmimo_gram_exact_noalloc, the array's only user)
  c->scratch_init = static_scratch_init(device);
  if (c->scratch_init != hipSuccess) (void)hipGetLastError();
  std::vector<double> gl, gl_f;
  c->n_gl = 64;
  gauss_legendre(c->n_gl, gl);
  gauss_legendre(kFresnelNodes, gl_f);
  gl.insert(gl.end(), gl_f.begin(), gl_f.end());
  if (hipMalloc(&c->d_gl, sizeof(double) * gl.size()) != hipSuccess ||
      hipMemcpy(c->d_gl, gl.data(), sizeof(double) * gl.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(c->d_counter);
    delete c;
    return XLMIMO_EDEVICE;
  }
  *out = c;
  return XLMIMO_OK;
}

int xlmimo_ctx_destroy(xlmimo_ctx* c) {
  if (!c) return XLMIMO_OK;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->capturing || c->graphs > 0) return set_err(c, XLMIMO_EINVAL, "destroy the context's graphs first");
  }
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (void* p : c->retired) (void)hipFree(p);
  for (auto& kv : c->plans) drop_plan_buffers(c, kv.second);   // no graphs: frees at once
  for (auto& kv : c->row_plans) drop_plan_buffers(c, kv.second);
  DevBuf* bufs[] = {&c->partials, &c->scratch_gram, &c->scratch_gram2, &c->scratch_rates, &c->scratch_bounds,
                    &c->scratch_nlist, &c->scratch_pairs, &c->scratch_routes, &c->scratch_vpos,
                    &c->scratch_vgram, &c->scratch_work};
  for (DevBuf* b : bufs)
    if (b->p) (void)hipFree(b->p);
  (void)hipFree(c->d_counter);
  (void)hipFree(c->d_gl);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
  return XLMIMO_OK;
}

const char* xlmimo_last_error(const xlmimo_ctx* c) { return c ? c->err.c_str() : "no context"; }

int xlmimo_timing_enable(xlmimo_ctx* c, int on) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  c->timing = on != 0;
  c->ev_used = 0;
  return XLMIMO_OK;
}

int xlmimo_timing_read(xlmimo_ctx* c, double* total_ms, int64_t* n_launches) {
  if (!c || !total_ms || !n_launches) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = no_capture(c, "xlmimo_timing_read")) return rc0;
  double tot = 0.0;
  for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
    HIP_TRY(c, hipEventSynchronize(c->ev_pool[i + 1]));
    float ms = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_pool[i], c->ev_pool[i + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *n_launches = (int64_t)(c->ev_used / 2);
  c->ev_used = 0;
  return XLMIMO_OK;
}

int xlmimo_gram_exact(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, int32_t precision,
                      double* gram_out, void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = stream_ok(c, stream)) return rc0;
  int rc = check_array(c, a);
  if (!rc) rc = check_batch(c, b, true, XLMIMO_MAX_USERS_EXACT);
  if (rc) return rc;
  if (precision != XLMIMO_FP64 && precision != XLMIMO_FP32C && precision != XLMIMO_FP32H)
    return set_err(c, XLMIMO_EINVAL, "bad precision %d", precision);
  if (b->n_drops == 0) return XLMIMO_OK;
  if (!gram_out) return set_err(c, XLMIMO_EINVAL, "gram_out is NULL");
  if ((rc = set_device(c))) return rc;
  return gram_exact_impl(c, a, b, nullptr, precision, gram_out, (hipStream_t)stream);
}

int xlmimo_gram_exact_noalloc(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, int32_t precision,
                              double* gram_out, void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  int rc = check_array(c, a);
  if (!rc) rc = check_batch(c, b, true, XLMIMO_MAX_USERS);
  if (rc) return rc;
  if (precision != XLMIMO_FP64 && precision != XLMIMO_FP32C && precision != XLMIMO_FP32H)
    return set_err(c, XLMIMO_EINVAL, "bad precision %d", precision);
  if (b->n_drops == 0) return XLMIMO_OK;
  if (!gram_out) return set_err(c, XLMIMO_EINVAL, "gram_out is NULL");
  if ((rc = set_device(c))) return rc;
  return gram_exact_noalloc_impl(c, a, b, precision, gram_out, (hipStream_t)stream);
}

int xlmimo_gram_update_users(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, int32_t precision,
                             int64_t n_moved, const int64_t* moved, double* gram_inout, void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = stream_ok(c, stream)) return rc0;
  int rc = check_array(c, a);
  if (!rc) rc = check_batch(c, b, true, XLMIMO_MAX_USERS_EXACT);
  if (rc) return rc;
  if (precision != XLMIMO_FP64 && precision != XLMIMO_FP32C && precision != XLMIMO_FP32H)
    return set_err(c, XLMIMO_EINVAL, "bad precision %d", precision);
  if (n_moved < 0) return set_err(c, XLMIMO_EINVAL, "n_moved must be >= 0");
  if (n_moved == 0 || b->n_drops == 0) return XLMIMO_OK;
  if (!moved || !gram_inout) return set_err(c, XLMIMO_EINVAL, "moved and gram_inout are required");
  int64_t total = 0;
  for (int64_t d = 0; d < b->n_drops; ++d) total += b->n_users[d];
  for (int64_t q = 0; q < n_moved; ++q) {
    if (moved[q] < 0 || moved[q] >= total)
      return set_err(c, XLMIMO_EINVAL, "moved[%lld] = %lld outside 0..%lld", (long long)q, (long long)moved[q],
                     (long long)(total - 1));
    if (q && moved[q] <= moved[q - 1]) return set_err(c, XLMIMO_EINVAL, "moved must be strictly ascending");
  }
  if ((rc = set_device(c))) return rc;
  Plan* p = nullptr;
  if ((rc = get_row_plan(c, a, b, n_moved, moved, &p))) return rc;
  return run_exact(c, a, b, p, precision, gram_inout, (hipStream_t)stream);
}

int xlmimo_cholesky(xlmimo_ctx* c, const xlmimo_batch* b, const double* gram, const double* rho,
                    double* factor_out, double* logdet_out, int32_t* status_out, void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = stream_ok(c, stream)) return rc0;
  int rc = check_batch(c, b, false, XLMIMO_MAX_USERS_EXACT);
  if (rc) return rc;
  if (b->n_drops == 0) return XLMIMO_OK;
  if (!gram || !factor_out) return set_err(c, XLMIMO_EINVAL, "gram and factor_out are required");
  if ((rc = set_device(c))) return rc;
  xlmimo_array dummy = {XLMIMO_ULA, XLMIMO_AMP_FREESPACE, 1, 1, 1.0, 1.0, 1.0};
  xlmimo_batch bb = *b;
  bb.n_elems = nullptr;
  Plan* p = nullptr;
  if ((rc = get_plan(c, &dummy, &bb, nullptr, &p))) return rc;
  HIP_TRY(c, launch_cholesky(p->d_drops, p->n_drops, gram, rho, factor_out, logdet_out, status_out,
                             (hipStream_t)stream));
  return XLMIMO_OK;
}

int xlmimo_cholesky_update_users(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, int64_t n_moved,
                                 const int64_t* moved, const double* gram, const double* rho, double* factor_inout,
                                 double* logdet_out, int32_t* status_out, void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = stream_ok(c, stream)) return rc0;
  int rc = check_array(c, a);
  if (!rc) rc = check_batch(c, b, false, XLMIMO_MAX_USERS_EXACT);
  if (rc) return rc;
  if (n_moved < 0) return set_err(c, XLMIMO_EINVAL, "n_moved must be >= 0");
  if (n_moved == 0 || b->n_drops == 0) return XLMIMO_OK;
  if (!moved || !gram || !factor_inout) return set_err(c, XLMIMO_EINVAL, "moved, gram and factor_inout are required");
  int64_t total = 0;
  for (int64_t d = 0; d < b->n_drops; ++d) total += b->n_users[d];
  for (int64_t q = 0; q < n_moved; ++q) {
    if (moved[q] < 0 || moved[q] >= total)
      return set_err(c, XLMIMO_EINVAL, "moved[%lld] = %lld outside 0..%lld", (long long)q, (long long)moved[q],
                     (long long)(total - 1));
    if (q && moved[q] <= moved[q - 1]) return set_err(c, XLMIMO_EINVAL, "moved must be strictly ascending");
  }
  if ((rc = set_device(c))) return rc;
  Plan* rp = nullptr;
  if ((rc = get_row_plan(c, a, b, n_moved, moved, &rp))) return rc;
  xlmimo_array dummy = {XLMIMO_ULA, XLMIMO_AMP_FREESPACE, 1, 1, 1.0, 1.0, 1.0};
  xlmimo_batch bb = *b;
  bb.n_elems = nullptr;
  Plan* p = nullptr;
  if ((rc = get_plan(c, &dummy, &bb, nullptr, &p))) return rc;
  HIP_TRY(c, launch_chol_update(p->d_drops, rp->n_mdrop, rp->d_mdrop, rp->d_moff, rp->d_mloc, gram, rho,
                                factor_inout, logdet_out, status_out, (hipStream_t)stream));
  return XLMIMO_OK;
}

int xlmimo_gram_closedform(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, int32_t variant,
                           double* gram_out, int32_t* status_out, void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = stream_ok(c, stream)) return rc0;
  int rc = check_array(c, a);
  if (!rc) rc = check_batch(c, b, true);
  if (rc) return rc;
  if (variant < XLMIMO_CF_PAPER || variant > XLMIMO_CF_GATED_QUAD) return set_err(c, XLMIMO_EINVAL, "bad variant %d", variant);
  if (variant >= XLMIMO_CF_UNIFORM && a->geometry != XLMIMO_ULA)
    return set_err(c, XLMIMO_EINVAL, "closed-form variant %d is defined for a ULA", variant);
  if (b->n_drops == 0) return XLMIMO_OK;
  if (!gram_out) return set_err(c, XLMIMO_EINVAL, "gram_out is NULL");
  if ((rc = set_device(c))) return rc;
  return closedform_impl(c, a, b, nullptr, variant, gram_out, status_out, (hipStream_t)stream);
}

static int check_rates_args(xlmimo_ctx* c, const xlmimo_batch* b, const double* gram_true, const double* gram_filter,
                            int32_t n_snr, const double* rho, int32_t schemes, int max_k = XLMIMO_MAX_USERS_EXACT) {
  int rc = check_batch(c, b, false, max_k);
  if (rc) return rc;
  if (schemes <= 0 || schemes > 127) return set_err(c, XLMIMO_EINVAL, "bad scheme mask %d", schemes);
  if (schemes & (XLMIMO_MZF | XLMIMO_MZF_MISM))
    for (int64_t d = 0; d < b->n_drops; ++d)
      if (b->n_users[d] > XLMIMO_MAX_USERS)
        return set_err(c, XLMIMO_EINVAL, "drop %lld: modified-ZF schemes take K <= %d", (long long)d,
                       XLMIMO_MAX_USERS);
  if (n_snr < 1) return set_err(c, XLMIMO_EINVAL, "n_snr must be >= 1");
  if (b->n_drops == 0) return XLMIMO_OK;
  if (!gram_true || !rho) return set_err(c, XLMIMO_EINVAL, "gram_true and rho are required");
  if ((schemes & (XLMIMO_MZF | XLMIMO_MZF_MISM)) && !gram_filter)
    return set_err(c, XLMIMO_EINVAL, "modified-ZF schemes need gram_filter");
  return XLMIMO_OK;
}

int xlmimo_zf_mmse_sumrate(xlmimo_ctx* c, const xlmimo_batch* b, const double* gram_true, const double* gram_filter,
                           int32_t n_snr, const double* rho, int32_t schemes, double* rates_out, int32_t* status_out,
                           void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = stream_ok(c, stream)) return rc0;
  int rc = check_rates_args(c, b, gram_true, gram_filter, n_snr, rho, schemes);
  if (rc) return rc;
  if (b->n_drops == 0) return XLMIMO_OK;
  if (!rates_out) return set_err(c, XLMIMO_EINVAL, "rates_out is NULL");
  if ((rc = set_device(c))) return rc;
  xlmimo_array dummy = {XLMIMO_ULA, XLMIMO_AMP_FREESPACE, 1, 1, 1.0, 1.0, 1.0};
  xlmimo_batch bb = *b;
  bb.n_elems = nullptr;
  Plan* p = nullptr;
  if ((rc = get_plan(c, &dummy, &bb, nullptr, &p))) return rc;
  double* work = nullptr;
  if ((rc = ensure_rates_work(c, p, (hipStream_t)stream, &work))) return rc;
  HIP_TRY(c, launch_rates(p->d_drops, p->n_drops, rates_k_max(p->k_max), gram_true, gram_filter, n_snr, rho,
                          p->total_users, schemes, rates_out, status_out, (hipStream_t)stream, work));
  return XLMIMO_OK;
}

int xlmimo_capacity_sweep(xlmimo_ctx* c, const xlmimo_array* a, int32_t n_N, const int64_t* N_list,
                          const xlmimo_batch* b, int32_t form, xlmimo_mlp* mlp, double log_var_max, int32_t n_snr,
                          const double* rho, int32_t schemes, double t_sat, double eps_sat, double* ergodic_out,
                          double* sat_out, int32_t* status_out, void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (int rc0 = stream_ok(c, stream)) return rc0;
  hipStream_t s = (hipStream_t)stream;
  int rc = check_array(c, a);
  if (rc) return rc;
  if (a->geometry != XLMIMO_ULA) return set_err(c, XLMIMO_EINVAL, "the capacity sweep varies a ULA's N");
  if (form < XLMIMO_FORM_EXACT_FP64 || form > XLMIMO_FORM_CF_UNIFORM) return set_err(c, XLMIMO_EINVAL, "bad form %d", form);
  if (form == XLMIMO_FORM_CF_GATED_MLP && (!mlp || mlp->ctx != c)) return set_err(c, XLMIMO_EINVAL, "the MLP form needs an mlp of this context");
  if (n_N < 1 || !N_list) return set_err(c, XLMIMO_EINVAL, "N_list is empty");
  for (int i = 0; i < n_N; ++i) {
    if (N_list[i] < 1 || N_list[i] > 2147483647LL) return set_err(c, XLMIMO_EINVAL, "N_list[%d] out of range", i);
    if (i && N_list[i] <= N_list[i - 1]) return set_err(c, XLMIMO_EINVAL, "N_list must be strictly ascending");
  }
  if (!(t_sat > 0.0 && t_sat < 1.0)) return set_err(c, XLMIMO_EINVAL, "t_sat must lie in (0, 1)");
  if (!(eps_sat >= 0.0 && eps_sat < 1.0)) return set_err(c, XLMIMO_EINVAL, "eps_sat must lie in [0, 1)");
  const bool cf = (form >= XLMIMO_FORM_CF_PAPER && form <= XLMIMO_FORM_CF_GATED_MLP) || form == XLMIMO_FORM_CF_UNIFORM;
  if (!cf && (schemes & (XLMIMO_MZF | XLMIMO_MZF_MISM)))
    return set_err(c, XLMIMO_EINVAL, "modified-ZF schemes need a closed-form sweep");
  if ((rc = check_rates_args(c, b, (const double*)1, (const double*)1, n_snr, rho, schemes,
                              cf ? XLMIMO_MAX_USERS : XLMIMO_MAX_USERS_EXACT)))
    return rc;
  if (!b->user_pos && b->n_drops) return set_err(c, XLMIMO_EINVAL, "user_pos is NULL");
  if (b->n_drops == 0) return XLMIMO_OK;
  if (!ergodic_out || !sat_out) return set_err(c, XLMIMO_EINVAL, "ergodic_out and sat_out are required");
  if ((rc = set_device(c))) return rc;

  const int n_sch = __builtin_popcount(schemes);
  const int n_vals = n_snr * n_sch;
  const int nd = (int)b->n_drops;
  Plan* p = nullptr;
  int64_t n0 = N_list[0];
  if ((rc = get_plan(c, a, b, &n0, &p))) return rc;
  const int64_t gbytes = sizeof(double) * 2 * p->gram_elems;
  if ((rc = ensure(c, c->scratch_gram, gbytes, s))) return rc;
  const bool need_exact_true = cf && (schemes & XLMIMO_MZF_MISM);
  if (need_exact_true && (rc = ensure(c, c->scratch_gram2, gbytes, s))) return rc;
  double* work = nullptr;
  if ((rc = ensure_rates_work(c, p, s, &work))) return rc;
  if ((rc = ensure(c, c->scratch_rates, sizeof(double) * (size_t)nd * n_vals, s))) return rc;
  if ((rc = ensure(c, c->scratch_bounds, sizeof(double) * 2 * (size_t)nd, s))) return rc;
  if (c->scratch_nlist.n < sizeof(double) * n_N) c->nlist_host.clear();
  if ((rc = ensure(c, c->scratch_nlist, sizeof(double) * n_N, s))) return rc;
  std::vector<double> nl(N_list, N_list + n_N);
  if (nl != c->nlist_host) {
    // synchronous upload, skipped when the list is unchanged (so a warmed-up sweep can be graph-captured)
    if (c->capturing)
      return set_err(c, XLMIMO_EINVAL, "a new N list needs an upload during graph capture: "
                     "run the same sweep once before capturing it");
    HIP_TRY(c, hipStreamSynchronize(s));
    HIP_TRY(c, hipMemcpy(c->scratch_nlist.p, nl.data(), sizeof(double) * n_N, hipMemcpyHostToDevice));
    c->nlist_host = nl;
  }

  double* g = (double*)c->scratch_gram.p;
  double* g2 = (double*)c->scratch_gram2.p;
  for (int i = 0; i < n_N; ++i) {
    int32_t* fb_flags = nullptr;
    const int64_t nn = N_list[i];
    int32_t* st = status_out ? status_out + (int64_t)i * nd : nullptr;
    if (!cf) {
      const int prec = form == XLMIMO_FORM_EXACT_FP64 ? XLMIMO_FP64
                       : (form == XLMIMO_FORM_EXACT_FP32H ? XLMIMO_FP32H : XLMIMO_FP32C);
      if ((rc = gram_exact_impl(c, a, b, &nn, prec, g, s))) return rc;
    } else {
      const int variant = form == XLMIMO_FORM_CF_PAPER     ? XLMIMO_CF_PAPER
                          : form == XLMIMO_FORM_CF_UNIFORM ? XLMIMO_CF_UNIFORM
                          : form == XLMIMO_FORM_CF_GATED   ? XLMIMO_CF_GATED
                                                           : XLMIMO_CF_GATED_QUAD;
      if (form == XLMIMO_FORM_CF_GATED_MLP) {
        if ((rc = closedform_mlp_impl(c, a, b, &nn, variant, mlp, log_var_max, g, nullptr, s, &fb_flags))) return rc;
      } else if ((rc = closedform_impl(c, a, b, &nn, variant, g, nullptr, s))) {
        return rc;
      }
      // the true channel of the mismatched scheme: FP64 (G~^-1 G amplifies the true Gram's error by
      // the condition number when the filter is accurate)
      if (need_exact_true && (rc = gram_exact_impl(c, a, b, &nn, XLMIMO_FP64, g2, s))) return rc;
    }
    if ((rc = get_plan(c, a, b, &nn, &p))) return rc;
    const double* gtrue = need_exact_true ? g2 : g;
    HIP_TRY(c, launch_rates(p->d_drops, nd, rates_k_max(p->k_max), gtrue, g, n_snr, rho, p->total_users, schemes,
                            (double*)c->scratch_rates.p, st, s, work));
    if (st && fb_flags) HIP_TRY(c, launch_or_flags(st, fb_flags, nd, XLMIMO_ST_FELL_BACK, s));
    HIP_TRY(c, launch_ergodic((double*)c->scratch_rates.p, nd, n_vals, ergodic_out + (int64_t)i * n_vals, s));
  }
  HIP_TRY(c, launch_y_bounds(b->user_pos, p->d_drops, nd, a->geometry, t_sat, (double*)c->scratch_bounds.p, s));
  HIP_TRY(c, launch_saturation((double*)c->scratch_bounds.p, nd, ergodic_out, (double*)c->scratch_nlist.p, n_N, n_vals,
                               a->spacing_m, eps_sat, sat_out, s));
  return XLMIMO_OK;
}


// ---- graph capture --------------------------------------------------------

int xlmimo_graph_begin(xlmimo_ctx* c, void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->capturing) return set_err(c, XLMIMO_EINVAL, "a graph capture is already open on this context");
  if (!stream) return set_err(c, XLMIMO_EINVAL, "graph capture needs a created (non-default) stream");
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
  c->capturing = true;
  c->cap_failed = false;
  c->cap_stream = (hipStream_t)stream;
  return XLMIMO_OK;
}

int xlmimo_graph_end(xlmimo_ctx* c, void* stream, xlmimo_graph** out) {
  if (!c || !out) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  *out = nullptr;
  if (!c->capturing || (hipStream_t)stream != c->cap_stream)
    return set_err(c, XLMIMO_EINVAL, "no graph capture is open on this stream");
  c->capturing = false;
  c->cap_stream = nullptr;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture((hipStream_t)stream, &g);
  if (e != hipSuccess || !g || c->cap_failed) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    const bool failed = c->cap_failed;
    c->cap_failed = false;
    return set_err(c, XLMIMO_EINVAL, "graph capture failed: %s",
                   failed ? "a call made during the capture returned an error" : hipGetErrorString(e));
  }
  size_t n_nodes = 0;
  (void)hipGraphGetNodes(g, nullptr, &n_nodes);
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) return set_err(c, XLMIMO_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
  xlmimo_graph* G = new xlmimo_graph();
  G->ctx = c;
  G->exec = ex;
  G->n_nodes = n_nodes;
  c->graphs += 1;
  *out = G;
  return XLMIMO_OK;
}

int xlmimo_graph_launch(xlmimo_graph* G, void* stream) {
  if (!G) return XLMIMO_EINVAL;
  xlmimo_ctx* c = G->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->capturing) return set_err(c, XLMIMO_EINVAL, "cannot launch a graph while a capture is open");
  int rc = set_device(c);
  if (rc) return rc;
  HIP_TRY(c, hipGraphLaunch(G->exec, (hipStream_t)stream));
  return XLMIMO_OK;
}

int64_t xlmimo_graph_node_count(const xlmimo_graph* G) { return G ? (int64_t)G->n_nodes : -1; }

int xlmimo_graph_destroy(xlmimo_graph* G) {
  if (!G) return XLMIMO_OK;
  xlmimo_ctx* c = G->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();  // a replay may still be running
  (void)hipGraphExecDestroy(G->exec);
  c->graphs -= 1;
  delete G;
  return XLMIMO_OK;
}

// ---- autotuner --------------------------------------------------------------

int xlmimo_autotune_exact(xlmimo_ctx* c, const xlmimo_array* a, const xlmimo_batch* b, int64_t n_elems,
                          int32_t precision, int64_t* chunk_out, int32_t* grid_out, double* ms_out, void* stream) {
  if (!c) return XLMIMO_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  int rc = no_capture(c, "xlmimo_autotune_exact");
  if (!rc) rc = check_array(c, a);
  if (!rc) rc = check_batch(c, b, true);
  if (rc) return rc;
  if (precision != XLMIMO_FP64 && precision != XLMIMO_FP32C && precision != XLMIMO_FP32H)
    return set_err(c, XLMIMO_EINVAL, "bad precision %d", precision);
  if (n_elems < 0 || n_elems > 2147483647LL) return set_err(c, XLMIMO_EINVAL, "bad n_elems");
  if (n_elems > 0 && a->geometry != XLMIMO_ULA) return set_err(c, XLMIMO_EINVAL, "n_elems overrides a ULA's N only");
  if (b->n_drops == 0) return XLMIMO_OK;
  if ((rc = set_device(c))) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int64_t* nov = n_elems > 0 ? &n_elems : nullptr;
  const uint64_t key = plan_key(a, b, nov);
  const uint64_t gkey = key ^ (uint64_t)precision;
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  const bool timing = c->timing;
  c->timing = false;
  auto rebuild = [&](Plan** p) -> int {
    auto it = c->plans.find(key);
    if (it != c->plans.end()) {
      HIP_TRY(c, hipStreamSynchronize(s));
      drop_plan_buffers(c, it->second);
      c->plans.erase(it);
    }
    return get_plan(c, a, b, nov, p);
  };
  // median of 3 timed launches after one warm-up
  auto time_it = [&](double* ms) -> int {
    Plan* p = nullptr;
    int r = get_plan(c, a, b, nov, &p);
    if (r) return r;
    if ((r = ensure(c, c->scratch_gram, sizeof(double) * 2 * std::max<int64_t>(p->gram_elems, 1), s))) return r;
    double t[3];
    for (int k = 0; k < 4; ++k) {
      HIP_TRY(c, hipEventRecord(e0, s));
      if ((r = gram_exact_impl(c, a, b, nov, precision, (double*)c->scratch_gram.p, s))) return r;
      HIP_TRY(c, hipEventRecord(e1, s));
      HIP_TRY(c, hipEventSynchronize(e1));
      float f = 0.0f;
      HIP_TRY(c, hipEventElapsedTime(&f, e0, e1));
      if (k) t[k - 1] = f;
    }
    std::sort(t, t + 3);
    *ms = t[1];
    return XLMIMO_OK;
  };
  c->tuned_grid.erase(gkey);
  double best = 1e300;
  int64_t best_chunk = 0;
  int last_items = -1;
  for (int64_t ch = 1024; ch <= 131072 && !rc; ch *= 2) {
    c->tuned_chunk[key] = ch;
    Plan* p = nullptr;
    if ((rc = rebuild(&p))) break;
    if (p->n_items == last_items) continue;  // same work list as the previous candidate
    last_items = p->n_items;
    double ms = 0.0;
    if ((rc = time_it(&ms))) break;
    if (ms < best) {
      best = ms;
      best_chunk = ch;
    }
  }
  Plan* p = nullptr;
  if (!rc) {
    c->tuned_chunk[key] = best_chunk;
    rc = rebuild(&p);
  }
  int best_grid = 0;
  if (!rc) {
    const int g0 = precision == XLMIMO_FP64 ? p->grid_fp64 : (precision == XLMIMO_FP32H ? p->grid_fp32h : p->grid_fp32);
    best_grid = g0;
    const int cand[3] = {g0, (3 * g0) / 4, g0 / 2};
    double best_g = 1e300;
    for (int i = 0; i < 3 && !rc; ++i) {
      if (cand[i] < 1) continue;
      c->tuned_grid[gkey] = cand[i];
      double ms = 0.0;
      if ((rc = time_it(&ms))) break;
      if (ms < best_g) {
        best_g = ms;
        best_grid = cand[i];
      }
    }
    if (!rc) {
      c->tuned_grid[gkey] = best_grid;
      best = best_g;
    }
  }
  c->timing = timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    c->tuned_chunk.erase(key);
    c->tuned_grid.erase(gkey);
    return rc;
  }
  if (chunk_out) *chunk_out = best_chunk;
  if (grid_out) *grid_out = best_grid;
  if (ms_out) *ms_out = best;
  return XLMIMO_OK;
}

}  // extern "C"
