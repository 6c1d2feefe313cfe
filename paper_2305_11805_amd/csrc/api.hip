// C ABI of libnnpot: argument checks, workspace layout and the order of
// launches for each entry point.  Everything after the checks is enqueued on
// the caller's stream; no call allocates memory.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <algorithm>
#include <initializer_list>
#include <string>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.h"

namespace nnp {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local char g_err[512] = "";

static nn_status fail(nn_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

static nn_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(NN_E_HIP, "%s: %s", what, hipGetErrorString(e));
  return NN_OK;
}

// ---------------------------------------------------------------------------
// launch plans: the defaults, or the ones nn_autotune measured for a shape
// class (atom count within a factor of two, list entries per atom rounded
// to a multiple of four, descriptor sizes, MLP widths and mode)
// ---------------------------------------------------------------------------

struct PlanKey {
  int n_log2, row4, S, nt, nra, n_rad, h1, h2, mode;
  bool operator<(const PlanKey& o) const {
    return std::tie(n_log2, row4, S, nt, nra, n_rad, h1, h2, mode) <
           std::tie(o.n_log2, o.row4, o.S, o.nt, o.nra, o.n_rad, o.h1, o.h2, o.mode);
  }
};
static std::mutex g_pmu;
static std::map<PlanKey, LaunchPlan> g_plans;

// NN_AUTOTUNE_CACHE=<file>: the table persists across processes.  The file
// is read on the first lookup or tuning of the process and rewritten after
// each nn_autotune (its entries merged with the process's, the process's
// winning; written to a temporary file and renamed into place).  One entry
// per line of a JSON array:
//   {"key": [n_log2, row4, S, n_theta, n_rs_ang, n_rad, h1, h2, mode], "plan": [f, a, m]}
// Lines that do not parse, or whose plan is out of range, are skipped.  The
// cache is best effort: a file that cannot be read or written changes nothing
// but the speed.
static bool g_cache_loaded = false;

static const char* cache_path() {
  const char* e = getenv("NN_AUTOTUNE_CACHE");
  return (e && *e) ? e : nullptr;
}

static bool plan_valid(const LaunchPlan& q) {
  auto w = [](int v) { return v == 0 || v == 1 || v == 2 || v == 4; };
  return w(q.wpa_fwd) && w(q.wpa_adj) && (q.mlp_waves == 0 || q.mlp_waves == 1 || q.mlp_waves == 4 || q.mlp_waves == 8);
}

static void cache_read(const char* path, std::map<PlanKey, LaunchPlan>& into, bool overwrite) {
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    PlanKey k{};
    LaunchPlan q{};
    const int n = sscanf(line, " {\"key\": [%d, %d, %d, %d, %d, %d, %d, %d, %d], \"plan\": [%d, %d, %d]}", &k.n_log2,
                         &k.row4, &k.S, &k.nt, &k.nra, &k.n_rad, &k.h1, &k.h2, &k.mode, &q.wpa_fwd, &q.wpa_adj,
                         &q.mlp_waves);
    if (n != 12 || !plan_valid(q)) continue;
    if (overwrite) into[k] = q;
    else into.emplace(k, q);
  }
  fclose(f);
}

static void cache_load_locked() {
  if (g_cache_loaded) return;
  g_cache_loaded = true;
  if (const char* path = cache_path()) cache_read(path, g_plans, false);
}

static void cache_store_locked() {
  const char* path = cache_path();
  if (!path) return;
  std::map<PlanKey, LaunchPlan> all;
  cache_read(path, all, true);  // entries other processes wrote meanwhile
  for (const auto& kv : g_plans) all[kv.first] = kv.second;
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid());
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  bool ok = fprintf(f, "[\n") > 0;
  size_t left = all.size();
  for (const auto& kv : all) {
    const PlanKey& k = kv.first;
    const LaunchPlan& q = kv.second;
    ok = ok && fprintf(f, "{\"key\": [%d, %d, %d, %d, %d, %d, %d, %d, %d], \"plan\": [%d, %d, %d]}%s\n", k.n_log2,
                       k.row4, k.S, k.nt, k.nra, k.n_rad, k.h1, k.h2, k.mode, q.wpa_fwd, q.wpa_adj, q.mlp_waves,
                       --left ? "," : "") > 0;
  }
  ok = ok && fprintf(f, "]\n") > 0;
  ok = (fclose(f) == 0) && ok;
  if (!ok || rename(tmp.c_str(), path) != 0) remove(tmp.c_str());
}

static PlanKey plan_key(int64_t n_atoms, int64_t capacity, const DescConst& P, const nn_model* model, int mode) {
  PlanKey k{};
  int b = 0;
  for (int64_t v = n_atoms; v > 0; v >>= 1) ++b;
  k.n_log2 = b;
  k.row4 = n_atoms > 0 ? (int)(((capacity + n_atoms - 1) / n_atoms + 2) / 4) : 0;
  k.S = P.S;
  k.nt = P.n_theta;
  k.nra = P.n_rs_ang;
  k.n_rad = P.n_rad;
  k.h1 = model ? model->mlp[0].width[1] : 0;
  k.h2 = model ? model->mlp[0].width[2] : 0;
  k.mode = mode;
  return k;
}

// NNPOT_PLAN="f,a,m" in the environment forces a plan on every call (waves
// per atom of the forward and adjoint passes in {0 (packed), 1, 2, 4},
// waves per MLP tile in {4, 8}, or 1 for the row-block MLP): lets tests run
// each launch variant against the oracle.
static bool forced_plan(LaunchPlan* out) {
  const char* e = getenv("NNPOT_PLAN");
  if (!e || !*e) return false;
  int f = 0, a = 0, m = 0;
  if (sscanf(e, "%d,%d,%d", &f, &a, &m) != 3) return false;
  auto ok = [](int w) { return w == 0 || w == 1 || w == 2 || w == 4; };
  if (!ok(f) || !ok(a) || (m != 1 && m != 4 && m != 8)) return false;
  *out = LaunchPlan{f, a, m};
  return true;
}

static LaunchPlan plan_for(int64_t n_atoms, int64_t capacity, const DescConst& P, const nn_model* model, int mode) {
  LaunchPlan forced;
  if (forced_plan(&forced)) return forced;
  const PlanKey k = plan_key(n_atoms, capacity, P, model, mode);
  std::lock_guard<std::mutex> g(g_pmu);
  cache_load_locked();
  auto it = g_plans.find(k);
  return it != g_plans.end() ? it->second : plan_default(n_atoms, P, capacity);
}

// ---------------------------------------------------------------------------
// stage timing with HIP events
// ---------------------------------------------------------------------------

struct TimedLaunch {
  int stage;
  hipEvent_t a, b;
};
static std::mutex g_tmu;
static bool g_timing = false;
static std::vector<TimedLaunch> g_tl;
static std::vector<hipEvent_t> g_event_pool;

static hipEvent_t take_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets the launches of one stage on stream s when timing is on.
struct StageTimer {
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  StageTimer(int st, hipStream_t st_s) : stage(st), s(st_s) {
    std::lock_guard<std::mutex> g(g_tmu);
    if (!g_timing) return;
    a = take_event();
    b = take_event();
    if (a && b) (void)hipEventRecord(a, s);
  }
  ~StageTimer() {
    std::lock_guard<std::mutex> g(g_tmu);
    if (!(a && b)) return;
    (void)hipEventRecord(b, s);
    g_tl.push_back({stage, a, b});
  }
};

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------

struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * (n > 0 ? n : 1);
    return p;
  }
};

struct Layout {
  // neighbor build
  StructGeom* geom;
  int64_t *n_bins, *bin_base, *bin_count, *bin_start, *row_count, *count_off, *scan_tmp, *count_meta;
  int32_t *atom_bin, *bin_rank, *flag;
  int4* bin_m;
  double4* bin_x;
  uint64_t* row_keys;
  int64_t *key_loc, *cursor;
  int kslot;
  int64_t max_bins;
  // energy / forces
  float *G, *lam, *E_atom;
  float4* pg;
  int32_t* perm;
  int64_t *sp_cnt, *sp_off, *sp_start;
  __bf16* wb;  // BF16 weights, W then W^T per species and layer
  size_t wb_elems;
  // weight gradient: per-atom stash, per-atom weights, chunk partials
  float *st_a1, *st_d1, *st_a2, *st_d2, *w_atom, *partial;
  float *st_t1, *st_x1, *st_x2;  // the force term's extra stash (a1_dot, x1, x2)
  LayBuf lay;                    // stashes of the layer-by-layer MLP (other architectures)
  float *qeq_out, *qeq_seed;     // charge equilibration: network outputs and seeds [N][3]
  double* qeq_q;                 // and the charges [N]
  double* loss_partial;          // block sums of nn_loss
  float* jac;  // stored Jacobian (NN_STORE_JACOBIAN within the memory budget)
  size_t bytes;
};

static size_t model_param_floats(const nn_model* m) {
  size_t t = 0;
  if (!m) return 0;
  for (int s = 0; s < m->n_species; ++s)
    for (int l = 0; l < m->mlp[s].n_layers; ++l)
      t += ((size_t)m->mlp[s].width[l + 1] * m->mlp[s].width[l] + 127) / 128 * 128;
  return t;
}

// Depths and widths of the model as the kernels see them (no weights).
static ModelDev model_shape(const nn_model* m) {
  ModelDev d{};
  if (!m) return d;
  d.S = m->n_species;
  for (int s = 0; s < m->n_species && s < NN_MAX_SPECIES; ++s) {
    d.m[s].n_layers = m->mlp[s].n_layers;
    for (int l = 0; l <= NN_MAX_LAYERS; ++l) d.m[s].width[l] = m->mlp[s].width[l];
  }
  return d;
}

// True when the fused two-hidden-layer kernels take this model: every
// species has two hidden layers of the same compiled widths.
static bool model_fused(const nn_model* m) {
  if (!m || m->n_species < 1) return false;
  const nn_mlp& q0 = m->mlp[0];
  if (q0.n_layers != 3 || q0.width[3] != 1 || !mlp_supported(q0.width[1], q0.width[2])) return false;
  for (int s = 1; s < m->n_species; ++s) {
    const nn_mlp& q = m->mlp[s];
    if (q.n_layers != 3 || q.width[1] != q0.width[1] || q.width[2] != q0.width[2] || q.width[3] != 1) return false;
  }
  return true;
}

// The fused two-hidden-layer MLP with this plan's launch: the row-block
// kernel (FP32 or BF16) for plan value 1 where it takes the shape, else the
// tile kernel.
static void run_mlp(const MlpArgs& a, const nn_model* model, int mode, int64_t N, int waves, hipStream_t s) {
  const int h1 = model->mlp[0].width[1], h2 = model->mlp[0].width[2];
  if (waves == 1 && mode == 0 && mlp_rows_supported(h1, h2, a.D)) {
    launch_mlp_rows(a, h1, h2, N, s);
    return;
  }
  if (waves == 1 && mode != 0 && mlp_rows_bf_supported(h1, h2, a.D)) {
    launch_mlp_rows_bf(a, h1, h2, mode, N, s);
    return;
  }
  launch_mlp(a, h1, h2, mode, N, waves == 1 ? 0 : waves, s);
}

// Stashes of the layer-by-layer MLP: activations, act' and the adjoint of
// each hidden layer, and with `tangent` the tangent activations, act'' z_dot
// and the tangent adjoint.
static void carve_layers(Carver& c, int64_t N, const nn_model* model, bool tangent, LayBuf& b) {
  const ModelDev shape = model_shape(model);
  lay_stash_widths(shape, b.ld);
  for (int h = 1; h < NN_MAX_LAYERS; ++h) {
    if (!b.ld[h]) continue;
    const size_t n = (size_t)N * b.ld[h];
    b.a[h] = c.take<float>(n);
    b.s[h] = c.take<float>(n);
    b.d[h] = c.take<float>(n);
    if (tangent) {
      b.at[h] = c.take<float>(n);
      b.q[h] = c.take<float>(n);
      b.dt[h] = c.take<float>(n);
    }
  }
}

static Layout carve(void* ws, int64_t N, int32_t B, int64_t capacity, int64_t D, int S, const nn_model* model,
                    size_t jac_floats = 0) {
  Layout L{};
  Carver c{static_cast<char*>(ws)};
  L.max_bins = 8 * N + 64 * (int64_t)B + 1;
  const int64_t scan_n = std::max<int64_t>(std::max<int64_t>(N, L.max_bins),
                                           std::max<int64_t>((int64_t)B, (int64_t)NN_MAX_SPECIES * ((N + 63) / 64 + 1)));
  // first, so that every call's layout puts it at the same place
  L.loss_partial = c.take<double>(loss_partial_elems(N, B));
  L.geom = c.take<StructGeom>(B);
  L.n_bins = c.take<int64_t>(B + 1);
  L.bin_base = c.take<int64_t>(B + 1);
  L.bin_count = c.take<int64_t>(L.max_bins + 1);
  L.bin_start = c.take<int64_t>(L.max_bins + 1);
  L.bin_rank = c.take<int32_t>(N);
  L.bin_m = c.take<int4>(N);
  L.bin_x = c.take<double4>(N);
  L.kslot = row_key_slot(N, capacity);
  L.row_keys = c.take<uint64_t>((size_t)N * L.kslot + (L.kslot > 0 ? 2 * (size_t)capacity : 0));
  L.key_loc = c.take<int64_t>(N);
  L.cursor = c.take<int64_t>(1);
  L.atom_bin = c.take<int32_t>(4 * N);
  L.row_count = c.take<int64_t>(N + 1);
  L.count_off = c.take<int64_t>(N + 1);
  L.scan_tmp = c.take<int64_t>(scan_scratch_elems(scan_n));
  L.flag = c.take<int32_t>(4);
  L.count_meta = c.take<int64_t>(8);
  if (D > 0) {
    L.G = c.take<float>((size_t)N * D);
    L.lam = c.take<float>((size_t)N * D);
    L.E_atom = c.take<float>(N);
    L.pg = c.take<float4>(capacity);
    L.perm = c.take<int32_t>(N);
    const int64_t nblk = (N + 63) / 64 > 0 ? (N + 63) / 64 : 1;
    L.sp_cnt = c.take<int64_t>((size_t)S * nblk + 1);
    L.sp_off = c.take<int64_t>((size_t)S * nblk + 1);
    L.sp_start = c.take<int64_t>(NN_MAX_SPECIES + 1);
    L.wb_elems = 4 * model_param_floats(model);
    L.wb = c.take<__bf16>(L.wb_elems);
    if (model && !model_fused(model) && model->n_species > 0) {
      carve_layers(c, N, model, true, L.lay);
      L.w_atom = c.take<float>(N);
      L.partial = c.take<float>(lay_partial_floats(N, model_shape(model)));
      if (model->mlp[0].width[model->mlp[0].n_layers] == 3) {
        L.qeq_out = c.take<float>((size_t)3 * N);
        L.qeq_seed = c.take<float>((size_t)3 * N);
        L.qeq_q = c.take<double>(N);
      }
    } else if (model && model->n_species > 0 && model->mlp[0].n_layers == 3) {
      const int H1 = model->mlp[0].width[1], H2 = model->mlp[0].width[2];
      L.st_a1 = c.take<float>((size_t)N * H1);
      L.st_d1 = c.take<float>((size_t)N * H1);
      L.st_a2 = c.take<float>((size_t)N * H2);
      L.st_d2 = c.take<float>((size_t)N * H2);
      L.st_t1 = c.take<float>((size_t)N * H1);
      L.st_x1 = c.take<float>((size_t)N * H1);
      L.st_x2 = c.take<float>((size_t)N * H2);
      L.w_atom = c.take<float>(N);
      ModelDev md{};
      md.S = S;
      md.m[0].width[0] = (int)D;
      md.m[0].width[1] = H1;
      md.m[0].width[2] = H2;
      L.partial = c.take<float>(wgrad_partial_floats(N, S, md));
    }
  }
  L.jac = jac_floats ? c.take<float>(jac_floats) : nullptr;
  L.bytes = c.off + 256;
  return L;
}

// The part of the workspace an energy/force evaluation without a stored
// Jacobian uses, and nothing else (no list-build or weight-gradient pieces):
// the layout of nn_energy_forces_noalloc in the library's own scratch.
static Layout carve_lean(void* ws, int64_t N, int32_t B, int64_t capacity, int64_t D, int S, const nn_model* model) {
  Layout L{};
  Carver c{static_cast<char*>(ws)};
  const int64_t nblk = (N + 63) / 64 > 0 ? (N + 63) / 64 : 1;
  L.scan_tmp = c.take<int64_t>(scan_scratch_elems((int64_t)S * nblk + 1));
  L.G = c.take<float>((size_t)N * D);
  L.lam = c.take<float>((size_t)N * D);
  L.E_atom = c.take<float>(N);
  L.pg = c.take<float4>(capacity);
  L.perm = c.take<int32_t>(N);
  L.sp_cnt = c.take<int64_t>((size_t)S * nblk + 1);
  L.sp_off = c.take<int64_t>((size_t)S * nblk + 1);
  L.sp_start = c.take<int64_t>(NN_MAX_SPECIES + 1);
  L.wb_elems = 4 * model_param_floats(model);
  L.wb = c.take<__bf16>(L.wb_elems);
  if (!model_fused(model)) carve_layers(c, N, model, false, L.lay);
  L.bytes = c.off + 256;
  (void)B;
  return L;
}

// ---------------------------------------------------------------------------
// the library's own scratch, for callers that cannot allocate
// (nn_energy_forces_noalloc).  A file-scope device array: every GPU the
// library runs on holds one copy of it from the library's load until the
// process ends.  In host code `scratch` is only a stand-in for the symbol;
// the device address of each GPU's copy comes from hipGetSymbolAddress on
// that GPU and is the only handle host code passes on.
// ---------------------------------------------------------------------------

constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_smu;
static void* g_scratch_dev[kMaxDevices];

// The address of the current device's copy of `scratch` (looked up once per
// device, on the first call there).
static nn_status static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(NN_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(NN_E_HIP, "device %d beyond the %d the library tracks", dev, kMaxDevices);
  std::lock_guard<std::mutex> g(g_smu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail(NN_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return NN_OK;
}

// ---------------------------------------------------------------------------
// argument checks
// ---------------------------------------------------------------------------

static nn_status check_system(const nn_system* sys) {
  if (!sys) return fail(NN_E_INVALID, "sys is NULL");
  if (sys->n_atoms < 0 || sys->n_structs < 0) return fail(NN_E_INVALID, "negative sizes");
  if (sys->n_atoms > INT32_MAX - 1) return fail(NN_E_INVALID, "more than 2^31-2 atoms");
  if (sys->n_structs == 0 && sys->n_atoms > 0) return fail(NN_E_INVALID, "atoms but no structures");
  if (sys->n_atoms > 0 && (!sys->pos || !sys->species)) return fail(NN_E_INVALID, "pos/species is NULL");
  if (sys->n_structs > 0 && (!sys->atom_ptr || !sys->cell || !sys->pbc))
    return fail(NN_E_INVALID, "atom_ptr/cell/pbc is NULL");
  return NN_OK;
}

static nn_status check_nlist(const nn_nlist* nl, const nn_system* sys, bool need_entries) {
  if (!nl) return fail(NN_E_INVALID, "nl is NULL");
  if (!nl->offsets || !nl->meta) return fail(NN_E_INVALID, "nl->offsets/meta is NULL");
  if (need_entries && (!nl->nbr || !nl->shift || !nl->rev)) return fail(NN_E_INVALID, "nl->nbr/shift/rev is NULL");
  if (nl->capacity < 0 || nl->capacity > INT32_MAX) return fail(NN_E_INVALID, "capacity out of range");
  (void)sys;
  return NN_OK;
}

static nn_status make_desc_const(const nn_mbp_params* p, DescConst* out) {
  if (!p) return fail(NN_E_INVALID, "params is NULL");
  if (p->n_species < 1 || p->n_species > NN_MAX_SPECIES) return fail(NN_E_INVALID, "n_species must be 1..8");
  if (!(p->rc > 0.0) || !isfinite(p->rc)) return fail(NN_E_INVALID, "rc must be positive");
  if (p->n_rad < 1 || p->n_rad > kMaxRad) return fail(NN_E_UNSUPPORTED, "n_rad must be 1..%d", kMaxRad);
  if (!desc_supported(p->n_theta, p->n_rs_ang))
    return fail(NN_E_UNSUPPORTED, "angular bins %d x %d not compiled (n_theta in {4,8,16}, n_rs_ang in {4,8})",
                p->n_theta, p->n_rs_ang);
  if (p->kind != NN_DESC_MBP && p->kind != NN_DESC_BP) return fail(NN_E_INVALID, "unknown descriptor kind");
  const bool bp = p->kind == NN_DESC_BP;
  if (!p->rs_rad) return fail(NN_E_INVALID, "grid arrays are NULL");
  if (bp) {
    if (!p->bp_zeta || !p->bp_lambda || !p->bp_eta) return fail(NN_E_INVALID, "BP term arrays are NULL");
    for (int t = 0; t < p->n_theta; ++t) {
      const double z = p->bp_zeta[t];
      if (!(z >= 1.0 && z <= 64.0 && floor(z) == z)) return fail(NN_E_UNSUPPORTED, "BP zeta must be an integer in [1, 64]");
      if (p->bp_lambda[t] != 1.0 && p->bp_lambda[t] != -1.0) return fail(NN_E_INVALID, "BP lambda must be +1 or -1");
    }
    for (int q = 0; q < p->n_rs_ang; ++q)
      if (!(p->bp_eta[q] >= 0.0) || !isfinite(p->bp_eta[q])) return fail(NN_E_INVALID, "BP eta must be >= 0");
    if (!(p->eta_rad >= 0.0)) return fail(NN_E_INVALID, "eta must be >= 0");
  } else {
    if (!p->theta_s || !p->rs_ang) return fail(NN_E_INVALID, "grid arrays are NULL");
    if (!(p->zeta >= 1.0 && p->zeta <= 1024.0 && floor(p->zeta) == p->zeta))
      return fail(NN_E_UNSUPPORTED, "zeta must be an integer in [1, 1024]");
    if (!(p->eps >= 0.0) || !(p->eta_rad >= 0.0) || !(p->eta_ang >= 0.0))
      return fail(NN_E_INVALID, "eps and eta must be >= 0");
  }
  DescConst P{};
  P.S = p->n_species;
  P.n_rad = p->n_rad;
  P.n_theta = p->n_theta;
  P.n_rs_ang = p->n_rs_ang;
  P.D = (int)(p->n_rad * p->n_species + p->n_theta * p->n_rs_ang * p->n_species * (p->n_species + 1) / 2);
  P.zeta = bp ? 1 : (int)p->zeta;
  P.kind = p->kind;
  P.rc = (float)p->rc;
  P.eta_rad = (float)p->eta_rad;
  P.eta_ang = (float)p->eta_ang;
  P.eps_ang = (float)p->eps;
  P.pi_over_rc = (float)(M_PI / p->rc);
  P.half_pi_over_rc = (float)(0.5 * M_PI / p->rc);
  if (bp) {
    for (int t = 0; t < p->n_theta; ++t) {
      P.bp_zeta[t] = (int)p->bp_zeta[t];
      P.bp_lam[t] = (float)p->bp_lambda[t];
      P.bp_pref[t] = (float)ldexp(1.0, 2 - (int)p->bp_zeta[t]);  // 2 * 2^(1 - zeta): both orders of a pair
    }
    for (int q = 0; q < p->n_rs_ang; ++q) P.bp_eta[q] = (float)p->bp_eta[q];
    P.bp_zbits = 0;
    for (int t = 0; t < p->n_theta; ++t)
      while ((P.bp_zeta[t] >> P.bp_zbits) != 0) ++P.bp_zbits;
  } else {
    const double norm = 1.0 + sqrt(1.0 + p->eps);
    for (int t = 0; t < p->n_theta; ++t) {
      P.x_a[t] = (float)(cos(p->theta_s[t]) / norm);
      P.x_b[t] = (float)(sin(p->theta_s[t]) / norm);
    }
    P.x_c = (float)(1.0 / norm);
  }
  for (int k = 0; k < p->n_rad; ++k) {
    P.rs_rad[k] = (float)p->rs_rad[k];
    P.rs_rad_lo[k] = (float)(p->rs_rad[k] - (double)P.rs_rad[k]);
  }
  for (int q = 0; q < p->n_rs_ang && !bp; ++q) {
    P.rs_ang[q] = (float)p->rs_ang[q];
    P.rs_ang_lo[q] = (float)(p->rs_ang[q] - (double)P.rs_ang[q]);
  }
  P.rc64 = p->rc;
  P.half_pi_over_rc64 = 0.5 * M_PI / p->rc;
  P.pi_over_rc64 = M_PI / p->rc;
  *out = P;
  return NN_OK;
}

static nn_status check_model(const nn_model* m, const DescConst& P, int n_out = 1) {
  if (!m) return fail(NN_E_INVALID, "model is NULL");
  if (m->n_species != P.S) return fail(NN_E_INVALID, "model has %d species, descriptor %d", m->n_species, P.S);
  for (int s = 0; s < m->n_species; ++s) {
    const nn_mlp& q = m->mlp[s];
    const int L = q.n_layers;
    if (L < 2 || L > NN_MAX_LAYERS)
      return fail(NN_E_UNSUPPORTED, "species %d: %d weight layers (1 to %d hidden layers are supported)", s, L,
                  NN_MAX_LAYERS - 1);
    if (q.width[0] != P.D) return fail(NN_E_INVALID, "species %d: input width %d != D %d", s, q.width[0], P.D);
    if (q.width[L] != n_out) return fail(NN_E_INVALID, "species %d: output width must be %d", s, n_out);
    for (int l = 1; l < L; ++l)
      if (q.width[l] < 1 || q.width[l] > 4096)
        return fail(NN_E_UNSUPPORTED, "species %d: hidden width %d outside 1..4096", s, q.width[l]);
    for (int l = 0; l < L; ++l) {
      if (!q.W[l] || !q.b[l]) return fail(NN_E_INVALID, "species %d layer %d: NULL weights", s, l);
      if (q.act[l] < 0 || q.act[l] > 3) return fail(NN_E_INVALID, "bad activation code");
    }
    if (q.act[L - 1] != NN_ACT_LINEAR) return fail(NN_E_UNSUPPORTED, "output layer must be linear");
  }
  return NN_OK;
}

// BF16 MLP modes exist only for the fused kernels' shapes.
static nn_status check_mode(const nn_model* m, int32_t flags) {
  if ((flags & (NN_BF16_MLP | NN_BF16X3_MLP)) && !model_fused(m))
    return fail(NN_E_UNSUPPORTED, "BF16 MLP modes need two hidden layers of widths (64,32), (128,128) or (256,128) "
                                  "shared by all species; other networks run in FP32");
  return NN_OK;
}

// Floats of the stored Jacobian if these flags and budget ask for it, else 0.
static size_t jac_request(const DescConst& P, int64_t capacity, int32_t flags, size_t mem_budget) {
  if (!(flags & (NN_STORE_JACOBIAN | NN_REUSE_DESCRIPTORS))) return 0;
  const size_t n = jacobian_floats(P.n_rad, P.S, P.n_theta, P.n_rs_ang, capacity);
  return n * sizeof(float) <= mem_budget ? n : 0;
}

static int64_t dim_of(const nn_mbp_params* p) {
  return (int64_t)p->n_rad * p->n_species + (int64_t)p->n_theta * p->n_rs_ang * p->n_species * (p->n_species + 1) / 2;
}

static NbLaunch nb_launch(const nn_system* sys, const Layout& L, double radius, nn_nlist* nl, bool count_only) {
  NbLaunch n{};
  n.sys = sys;
  n.radius = radius;
  n.capacity = nl ? nl->capacity : 0;
  n.nl = nl;
  n.counts = L.row_count;
  n.offsets = count_only ? L.count_off : nl->offsets;
  n.geom = L.geom;
  n.n_bins = L.n_bins;
  n.bin_base = L.bin_base;
  n.bin_count = L.bin_count;
  n.bin_start = L.bin_start;
  n.bin_rank = L.bin_rank;
  n.bin_m = L.bin_m;
  n.bin_x = L.bin_x;
  n.row_keys = L.row_keys;
  n.key_loc = L.key_loc;
  n.cursor = L.cursor;
  n.kslot = L.kslot;
  n.atom_bin = L.atom_bin;
  n.scan_tmp = L.scan_tmp;
  n.flag = L.flag;
  n.meta = count_only ? L.count_meta : nl->meta;
  n.max_bins = L.max_bins;
  return n;
}

// Fill the kernels' view of the model; in BF16 modes also enqueue the BF16
// hi/lo weight copies into the workspace.
static void prepare_model(const nn_model* model, const DescConst& P, const Layout& L, bool bf16, MlpArgs& a,
                          hipStream_t s) {
  a.model.S = P.S;
  ConvJob job{};
  size_t wofs = 0;
  for (int sp = 0; sp < P.S; ++sp) {
    const nn_mlp& q = model->mlp[sp];
    MlpDev& d = a.model.m[sp];
    d.n_layers = q.n_layers;
    for (int l = 0; l <= q.n_layers; ++l) d.width[l] = q.width[l];
    for (int l = 0; l < q.n_layers; ++l) {
      d.act[l] = q.act[l];
      d.W[l] = q.W[l];
      d.b[l] = q.b[l];
    }
    if (bf16) {
      for (int l = 0; l < 2; ++l) {
        const size_t n = ((size_t)q.width[l + 1] * q.width[l] + 127) / 128 * 128;
        __bf16* w = L.wb + wofs;
        wofs += 4 * n;
        d.Wb[l] = w;
        d.Wl[l] = w + n;
        d.WbT[l] = w + 2 * n;
        d.WlT[l] = w + 3 * n;
        job.src[job.n] = q.W[l];
        job.hi[job.n] = w;
        job.lo[job.n] = w + n;
        job.hiT[job.n] = w + 2 * n;
        job.loT[job.n] = w + 3 * n;
        job.rows[job.n] = q.width[l + 1];
        job.cols[job.n] = q.width[l];
        ++job.n;
      }
    }
  }
  if (bf16) {
    StageTimer t(NN_STAGE_WEIGHTS, s);
    launch_convert_bf16(job, s);
  }
}

__global__ void k_zero_meta(int64_t* m) {
  if (threadIdx.x < 8) m[threadIdx.x] = 0;
}

// Records which build of the list the workspace's stored Jacobian belongs to.
__global__ void k_mark_jac(int64_t* meta) {
  if (threadIdx.x == 0) meta[kMetaJac] = meta[kMetaBuilds] + 1;
}

// Checks shared by the energy/force entry points; fills the kernels'
// descriptor constants.
static nn_status check_ef_args(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p, const nn_model* model,
                               int32_t flags, const double* E_struct, DescConst* P) {
  nn_status st = check_system(sys);
  if (st) return st;
  if ((st = check_nlist(nl, sys, true))) return st;
  if ((st = make_desc_const(p, P))) return st;
  if ((st = check_model(model, *P))) return st;
  if (!E_struct && sys->n_structs > 0) return fail(NN_E_INVALID, "E_struct is NULL");
  if (nl->radius < p->rc) return fail(NN_E_INVALID, "list radius %g < rc %g", nl->radius, p->rc);
  if (flags & ~(NN_BF16_MLP | NN_BF16X3_MLP | NN_STORE_JACOBIAN | NN_REUSE_DESCRIPTORS))
    return fail(NN_E_INVALID, "unknown flags");
  if ((flags & NN_BF16_MLP) && (flags & NN_BF16X3_MLP))
    return fail(NN_E_INVALID, "NN_BF16_MLP and NN_BF16X3_MLP are exclusive");
  return check_mode(model, flags);
}

// The layer-by-layer MLP's view of a fused-kernel argument block and the
// workspace.
static LayArgs lay_args(const MlpArgs& a, const Layout& L) {
  LayArgs la{};
  la.model = a.model;
  la.perm = a.perm;
  la.sp_start = a.sp_start;
  la.G = a.G;
  la.D = a.D;
  la.w_atom = L.w_atom;
  la.E_atom = a.E_atom;
  la.lambda = a.lambda ? a.lambda : L.lam;
  la.buf = L.lay;
  la.n_out = 1;
  return la;
}

// The launches of one energy/force evaluation on the workspace layout L
// (stored: the layout holds a Jacobian within the caller's budget).
static void ef_enqueue(const nn_system* sys, const nn_nlist* nl, const DescConst& P, const nn_model* model,
                       int32_t flags, const Layout& L, bool stored, double* E_struct, float* E_atom, float* F,
                       hipStream_t s) {
  const bool reuse = flags & NN_REUSE_DESCRIPTORS;
  const int64_t N = sys->n_atoms;
  const int mode = (flags & NN_BF16X3_MLP) ? 2 : (flags & NN_BF16_MLP) ? 1 : 0;
  const bool bf16 = mode != 0;
  if (N == 0) {
    if (sys->n_structs > 0) launch_energy_reduce(L.E_atom, sys->atom_ptr, sys->n_structs, N, E_struct, s);
    return;
  }
  const LaunchPlan plan = plan_for(N, nl->capacity, P, model, mode);
  // species grouping (with one species the descriptor launch writes the
  // identity grouping)
  const bool fold_species = P.S == 1 && !reuse;
  if (!fold_species) {
    StageTimer t(NN_STAGE_SPECIES, s);
    launch_species_group(sys->species, N, P.S, L.sp_cnt, L.sp_off, L.scan_tmp, L.perm, L.sp_start, s);
  }
  MlpArgs a{};
  prepare_model(model, P, L, bf16, a, s);
  // descriptors (and the stored Jacobian)
  if (!reuse) {
    StageTimer t(NN_STAGE_DESC_FWD, s);
    launch_desc_fwd(*sys, *nl, P, L.G, fold_species ? IdentityGroup{L.perm, L.sp_start} : IdentityGroup{},
                    plan.wpa_fwd, s);
  }
  if (stored && !reuse) {
    StageTimer t(NN_STAGE_DESC_JAC, s);
    launch_desc_jac(*sys, *nl, P, L.jac, s);
    hipLaunchKernelGGL(k_mark_jac, dim3(1), dim3(64), 0, s, nl->meta);
  }
  // MLP energies and lambda
  a.G = L.G;
  a.perm = L.perm;
  a.sp_start = L.sp_start;
  a.E_atom = E_atom ? E_atom : L.E_atom;
  a.lambda = F ? L.lam : nullptr;
  a.D = P.D;
  {
    StageTimer t(NN_STAGE_MLP, s);
    if (model_fused(model)) run_mlp(a, model, mode, N, plan.mlp_waves, s);
    else launch_mlp_layers(lay_args(a, L), N, F != nullptr, s);
  }
  if (!F) {
    StageTimer t(NN_STAGE_ENERGY, s);
    launch_energy_reduce(a.E_atom, sys->atom_ptr, sys->n_structs, N, E_struct, s);
  } else {
    if (stored) {
      StageTimer t(NN_STAGE_JAC_CONTRACT, s);
      launch_jac_contract(*sys, *nl, P, L.lam, L.jac, L.pg, s);
    } else {
      StageTimer t(NN_STAGE_DESC_ADJ, s);
      launch_desc_adj(*sys, *nl, P, L.lam, L.pg, plan.wpa_adj, s);
    }
    // the per-structure energy sums ride along in the gather's launch
    StageTimer t(NN_STAGE_FORCE_GATHER, s);
    launch_force_gather(*sys, *nl, L.pg, F, EnergyJob{a.E_atom, sys->atom_ptr, sys->n_structs, E_struct}, s);
  }
}

// Charge equilibration: the argument block of the solve and Coulomb kernels.
static nn_status make_qeq_args(const nn_system* sys, const nn_nlist* nl, const nn_qeq_params* qp, const DescConst& P,
                               const double* total_charge, double* E_struct, double* charges, const Layout& L,
                               QeqArgs* out) {
  if (!qp || !qp->sigma) return fail(NN_E_INVALID, "charge equilibration parameters are NULL");
  if (!(qp->coulomb > 0.0) || !isfinite(qp->coulomb)) return fail(NN_E_INVALID, "coulomb must be > 0");
  QeqArgs a{};
  for (int s = 0; s < P.S; ++s) {
    if (!(qp->sigma[s] > 0.0) || !isfinite(qp->sigma[s])) return fail(NN_E_INVALID, "sigma must be > 0");
    a.sigma[s] = qp->sigma[s];
  }
  if (sys->n_structs > 0 && (!total_charge || !E_struct)) return fail(NN_E_INVALID, "total_charge/E_struct is NULL");
  a.pos = sys->pos;
  a.species = sys->species;
  a.atom_ptr = sys->atom_ptr;
  a.pbc = sys->pbc;
  a.B = sys->n_structs;
  a.N = sys->n_atoms;
  a.out = L.qeq_out;
  a.total = total_charge;
  a.ke = qp->coulomb;
  a.E_struct = E_struct;
  a.q = charges ? charges : L.qeq_q;
  a.seed = L.qeq_seed;
  a.meta = nl->meta;
  *out = a;
  return NN_OK;
}

}  // namespace nnp

using namespace nnp;

extern "C" {

int64_t nn_descriptor_dim(const nn_mbp_params* p) {
  DescConst P;
  if (make_desc_const(p, &P) != NN_OK) return -1;
  return P.D;
}

nn_status nn_workspace_size(int64_t n_atoms, int32_t n_structs, int64_t capacity, const nn_mbp_params* p,
                            const nn_model* model, int32_t flags, size_t mem_budget, size_t* bytes) {
  if (!bytes) return fail(NN_E_INVALID, "bytes is NULL");
  if (n_atoms < 0 || n_structs < 0 || capacity < 0) return fail(NN_E_INVALID, "negative sizes");
  int64_t D = 0;
  int S = 1;
  size_t jf = 0;
  if (p) {
    DescConst P;
    nn_status st = make_desc_const(p, &P);
    if (st) return st;
    D = P.D;
    S = P.S;
    jf = jac_request(P, capacity, flags, mem_budget);
  }
  Layout L = carve(nullptr, n_atoms, n_structs, capacity, D, S, model, jf);
  *bytes = L.bytes;
  return NN_OK;
}

nn_status nn_count_neighbors(const nn_system* sys, double radius, int64_t* nnz, void* ws, size_t ws_bytes,
                             void* stream) {
  nn_status st = check_system(sys);
  if (st) return st;
  if (!nnz) return fail(NN_E_INVALID, "nnz is NULL");
  if (!(radius > 0.0)) return fail(NN_E_INVALID, "radius must be positive");
  Layout L = carve(nullptr, sys->n_atoms, sys->n_structs, 0, 0, 1, nullptr);
  if (!ws || ws_bytes < L.bytes) return fail(NN_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.bytes);
  L = carve(ws, sys->n_atoms, sys->n_structs, 0, 0, 1, nullptr);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_meta, dim3(1), dim3(64), 0, s, L.count_meta);
  NbLaunch nl = nb_launch(sys, L, radius, nullptr, true);
  launch_neighbors(nl, false, 0.0, true, s);
  if ((st = check_launch("nn_count_neighbors"))) return st;
  int64_t meta[8];
  if (hipMemcpyAsync(meta, L.count_meta, sizeof meta, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(NN_E_HIP, "nn_count_neighbors: %s", hipGetErrorString(hipGetLastError()));
  if (meta[kMetaErr] & kErrPtr) return fail(NN_E_INVALID, "atom_ptr must run from 0 to N without decreasing");
  if (meta[kMetaErr] & (kErrCell | kErrNonFinite | kErrShift | kErrTooMany))
    return fail(meta[kMetaErr] & kErrCell ? NN_E_CELL : NN_E_DEVICE, "neighbor count failed (error bits %lld)",
                (long long)meta[kMetaErr]);
  *nnz = meta[kMetaNnz];
  return NN_OK;
}

nn_status nn_build_neighbors(const nn_system* sys, double rc, double skin, nn_nlist* nl, void* ws, size_t ws_bytes,
                             void* stream) {
  nn_status st = check_system(sys);
  if (st) return st;
  if ((st = check_nlist(nl, sys, true))) return st;
  if (!(rc > 0.0) || !(skin >= 0.0)) return fail(NN_E_INVALID, "rc must be > 0 and skin >= 0");
  if (skin > 0.0 && !nl->ref_pos) return fail(NN_E_INVALID, "skin > 0 needs nl->ref_pos");
  Layout L = carve(nullptr, sys->n_atoms, sys->n_structs, nl->capacity, 0, 1, nullptr);
  if (!ws || ws_bytes < L.bytes) return fail(NN_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.bytes);
  L = carve(ws, sys->n_atoms, sys->n_structs, nl->capacity, 0, 1, nullptr);
  hipStream_t s = (hipStream_t)stream;
  NbLaunch nb = nb_launch(sys, L, rc + skin, nl, false);
  {
    StageTimer t(NN_STAGE_NEIGHBORS, s);
    launch_neighbors(nb, skin > 0.0, skin, false, s);
  }
  nl->radius = rc + skin;
  return check_launch("nn_build_neighbors");
}

nn_status nn_descriptors(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p, float* G, float* jac,
                         void* ws, size_t ws_bytes, void* stream) {
  nn_status st = check_system(sys);
  if (st) return st;
  if ((st = check_nlist(nl, sys, true))) return st;
  DescConst P;
  if ((st = make_desc_const(p, &P))) return st;
  if (!G && sys->n_atoms > 0) return fail(NN_E_INVALID, "G is NULL");

  if (nl->radius < p->rc) return fail(NN_E_INVALID, "list radius %g < rc %g", nl->radius, p->rc);
  (void)ws;
  (void)ws_bytes;
  hipStream_t s = (hipStream_t)stream;
  {
    StageTimer t(NN_STAGE_DESC_FWD, s);
    launch_desc_fwd(*sys, *nl, P, G, IdentityGroup{}, plan_for(sys->n_atoms, nl->capacity, P, nullptr, 0).wpa_fwd, s);
  }
  if (jac) {
    StageTimer t(NN_STAGE_DESC_JAC, s);
    launch_desc_jac(*sys, *nl, P, jac, s);
  }
  return check_launch("nn_descriptors");
}

nn_status nn_descriptor_tangent(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p, const float* v,
                                float* U, void* stream) {
  nn_status st = check_system(sys);
  if (st) return st;
  if ((st = check_nlist(nl, sys, true))) return st;
  DescConst P;
  if ((st = make_desc_const(p, &P))) return st;
  if ((!v || !U) && sys->n_atoms > 0) return fail(NN_E_INVALID, "v/U is NULL");
  if (nl->radius < p->rc) return fail(NN_E_INVALID, "list radius %g < rc %g", nl->radius, p->rc);
  hipStream_t s = (hipStream_t)stream;
  launch_desc_tan(*sys, *nl, P, v, U, plan_for(sys->n_atoms, nl->capacity, P, nullptr, 0).wpa_fwd, s);
  return check_launch("nn_descriptor_tangent");
}

nn_status nn_energy_forces(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p, const nn_model* model,
                           int32_t flags, size_t mem_budget, double* E_struct, float* E_atom, float* F, void* ws,
                           size_t ws_bytes, void* stream) {
  DescConst P;
  nn_status st = check_ef_args(sys, nl, p, model, flags, E_struct, &P);
  if (st) return st;
  const int64_t N = sys->n_atoms;
  const size_t jf = jac_request(P, nl->capacity, flags, mem_budget);
  if ((flags & NN_REUSE_DESCRIPTORS) && !jf)
    return fail(NN_E_INVALID, "NN_REUSE_DESCRIPTORS needs the stored Jacobian within mem_budget");
  Layout L = carve(nullptr, N, sys->n_structs, nl->capacity, P.D, P.S, model, jf);
  if (!ws || ws_bytes < L.bytes) return fail(NN_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.bytes);
  L = carve(ws, N, sys->n_structs, nl->capacity, P.D, P.S, model, jf);
  ef_enqueue(sys, nl, P, model, flags, L, jf != 0, E_struct, E_atom, F, (hipStream_t)stream);
  return check_launch("nn_energy_forces");
}

nn_status nn_energy_forces_noalloc(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p,
                                   const nn_model* model, int32_t flags, double* E_struct, float* E_atom, float* F,
                                   void* stream) {
  DescConst P;
  nn_status st = check_ef_args(sys, nl, p, model, flags, E_struct, &P);
  if (st) return st;
  if (flags & (NN_STORE_JACOBIAN | NN_REUSE_DESCRIPTORS))
    return fail(NN_E_INVALID, "nn_energy_forces_noalloc takes only the MLP precision flags");
  const int64_t N = sys->n_atoms;
  Layout L = carve_lean(nullptr, N, sys->n_structs, nl->capacity, P.D, P.S, model);
  if (L.bytes > kStaticScratchBytes)
    return fail(NN_E_WORKSPACE, "nn_energy_forces_noalloc: needs %zu bytes of scratch, the library holds %zu", L.bytes,
                kStaticScratchBytes);
  void* ws = nullptr;
  if ((st = static_scratch(&ws))) return st;
  L = carve_lean(ws, N, sys->n_structs, nl->capacity, P.D, P.S, model);
  ef_enqueue(sys, nl, P, model, flags, L, false, E_struct, E_atom, F, (hipStream_t)stream);
  return check_launch("nn_energy_forces_noalloc");
}

nn_status nn_autotune(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p, const nn_model* model,
                      int32_t flags, void* ws, size_t ws_bytes, void* stream, int32_t* plan_out) {
  nn_status st = check_system(sys);
  if (st) return st;
  if ((st = check_nlist(nl, sys, true))) return st;
  DescConst P;
  if ((st = make_desc_const(p, &P))) return st;
  if ((st = check_model(model, P))) return st;
  if ((st = check_mode(model, flags))) return st;
  if (nl->radius < p->rc) return fail(NN_E_INVALID, "list radius %g < rc %g", nl->radius, p->rc);
  if (flags & ~(NN_BF16_MLP | NN_BF16X3_MLP | NN_STORE_JACOBIAN | NN_REUSE_DESCRIPTORS))
    return fail(NN_E_INVALID, "unknown flags");
  if ((flags & NN_BF16_MLP) && (flags & NN_BF16X3_MLP))
    return fail(NN_E_INVALID, "NN_BF16_MLP and NN_BF16X3_MLP are exclusive");
  const int64_t N = sys->n_atoms;
  Layout L = carve(nullptr, N, sys->n_structs, nl->capacity, P.D, P.S, model);
  if (!ws || ws_bytes < L.bytes) return fail(NN_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.bytes);
  L = carve(ws, N, sys->n_structs, nl->capacity, P.D, P.S, model);
  const int mode = (flags & NN_BF16X3_MLP) ? 2 : (flags & NN_BF16_MLP) ? 1 : 0;
  LaunchPlan best = plan_default(N, P, nl->capacity);
  if (N > 0) {
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
      return fail(NN_E_HIP, "nn_autotune: event creation failed");
    launch_species_group(sys->species, N, P.S, L.sp_cnt, L.sp_off, L.scan_tmp, L.perm, L.sp_start, s);
    MlpArgs a{};
    prepare_model(model, P, L, mode != 0, a, s);
    a.G = L.G;
    a.perm = L.perm;
    a.sp_start = L.sp_start;
    a.E_atom = L.E_atom;
    a.lambda = L.lam;
    a.D = P.D;
    const int h1 = model->mlp[0].width[1], h2 = model->mlp[0].width[2];
    const bool fused = model_fused(model);
    // one pass of the step's three tuned stages under plan q, with events
    // around stage `which` (0 forward, 1 MLP, 2 adjoint; -1: none): each
    // candidate is timed where it runs in a step, after the stage before it
    // (timed back to back on its own, a launch overlapped the L2 state of the
    // previous one and the adjoint's choice came out 8 % slower in the step)
    auto step = [&](const LaunchPlan& q, int which) -> bool {
      auto mark = [&](int stage, hipEvent_t e) { return which != stage || hipEventRecord(e, s) == hipSuccess; };
      bool ok = mark(0, e0);
      launch_desc_fwd(*sys, *nl, P, L.G, IdentityGroup{}, q.wpa_fwd, s);
      ok = ok && mark(0, e1) && mark(1, e0);
      if (fused) run_mlp(a, model, mode, N, q.mlp_waves, s);
      else launch_mlp_layers(lay_args(a, L), N, true, s);
      ok = ok && mark(1, e1) && mark(2, e0);
      launch_desc_adj(*sys, *nl, P, L.lam, L.pg, q.wpa_adj, s);
      return ok && mark(2, e1);
    };
    // mean time of stage `which` over three steps after one untimed one; -1 on an error
    auto time_of = [&](const LaunchPlan& q, int which) -> float {
      if (!step(q, -1)) return -1.f;
      float tot = 0.f;
      for (int r = 0; r < 3; ++r) {
        float ms = -1.f;
        if (!step(q, which) || hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
          return -1.f;
        tot += ms;
      }
      return tot / 3.f;
    };
    // the fastest candidate for one stage (the others at their current
    // choice): two interleaved passes, each candidate's best time
    auto pick = [&](std::initializer_list<int> cands, auto&& usable, int which, int LaunchPlan::*field) {
      int wv[8];
      float tb[8];
      int n = 0;
      for (int w : cands)
        if (usable(w)) wv[n] = w, tb[n++] = -1.f;
      for (int pass = 0; pass < 2; ++pass)
        for (int c = 0; c < n; ++c) {
          LaunchPlan q = best;
          q.*field = wv[c];
          const float t = time_of(q, which);
          if (t >= 0.f && (tb[c] < 0.f || t < tb[c])) tb[c] = t;
        }
      float tbest = -1.f;
      for (int c = 0; c < n; ++c)
        if (tb[c] >= 0.f && (tbest < 0.f || tb[c] < tbest)) tbest = tb[c], best.*field = wv[c];
    };
    const bool pk = packed_supported(P) && nl->capacity <= 48 * N;  // rows short enough for any to be packed
    auto desc_ok = [&](int w) { return w != 0 || pk; };
    auto mlp_ok = [&](int w) {
      if (!fused) return w == best.mlp_waves;  // no launch choice for the layer-by-layer MLP
      if (w == 8) return h1 >= 128;
      if (w == 1) return mode == 0 ? mlp_rows_supported(h1, h2, P.D) : mlp_rows_bf_supported(h1, h2, P.D);
      return true;
    };
    pick({0, 1, 2, 4}, desc_ok, 0, &LaunchPlan::wpa_fwd);
    pick({4, 8, 1}, mlp_ok, 1, &LaunchPlan::mlp_waves);
    pick({0, 1, 2, 4}, desc_ok, 2, &LaunchPlan::wpa_adj);
    const bool destroyed = hipEventDestroy(e0) == hipSuccess && hipEventDestroy(e1) == hipSuccess;
    if ((st = check_launch("nn_autotune"))) return st;
    if (!destroyed) return fail(NN_E_HIP, "nn_autotune: event release failed");
    std::lock_guard<std::mutex> g(g_pmu);
    cache_load_locked();
    g_plans[plan_key(N, nl->capacity, P, model, mode)] = best;
    cache_store_locked();
  }
  if (plan_out) {
    plan_out[0] = best.wpa_fwd;
    plan_out[1] = best.wpa_adj;
    plan_out[2] = best.mlp_waves;
  }
  return NN_OK;
}

void nn_autotune_reset(void) {
  std::lock_guard<std::mutex> g(g_pmu);
  g_plans.clear();
  g_cache_loaded = true;  // the cache file is not read again by this process
}

nn_status nn_launch_plan(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p, const nn_model* model,
                         int32_t flags, int32_t* plan_out) {
  nn_status st = check_system(sys);
  if (st) return st;
  if ((st = check_nlist(nl, sys, false))) return st;
  DescConst P;
  if ((st = make_desc_const(p, &P))) return st;
  if ((st = check_model(model, P))) return st;
  if ((st = check_mode(model, flags))) return st;
  if (!plan_out) return fail(NN_E_INVALID, "plan_out is NULL");
  const int mode = (flags & NN_BF16X3_MLP) ? 2 : (flags & NN_BF16_MLP) ? 1 : 0;
  const LaunchPlan q = plan_for(sys->n_atoms, nl->capacity, P, model, mode);
  plan_out[0] = q.wpa_fwd;
  plan_out[1] = q.wpa_adj;
  plan_out[2] = q.mlp_waves;
  return NN_OK;
}

nn_status nn_energy_forces_grad(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p,
                                const nn_model* model, int32_t flags, const double* dL_dE, const float* dL_dF,
                                const float* F, float* dL_dpos, float* const* dW, float* const* db, void* ws,
                                size_t ws_bytes, void* stream) {
  nn_status st = check_system(sys);
  if (st) return st;
  if ((st = check_nlist(nl, sys, true))) return st;
  DescConst P;
  if ((st = make_desc_const(p, &P))) return st;
  if ((st = check_model(model, P))) return st;
  if (!dL_dF && (st = check_mode(model, flags))) return st;
  if (flags & ~(NN_BF16_MLP | NN_BF16X3_MLP | NN_STORE_JACOBIAN)) return fail(NN_E_INVALID, "unknown flags");
  if (!dL_dE && !dL_dF && sys->n_structs > 0) return fail(NN_E_INVALID, "dL_dE and dL_dF are both NULL");
  if (dL_dpos && dL_dF)
    return fail(NN_E_UNSUPPORTED, "the position gradient of a loss on forces (second derivatives) is not provided");
  if (dL_dpos && !dL_dE) return fail(NN_E_INVALID, "dL_dpos needs dL_dE");
  if (dL_dpos && !F) return fail(NN_E_INVALID, "dL_dpos needs the forces F");
  const int64_t N = sys->n_atoms;
  // the stored Jacobian (if any) sits after every piece used here, so the
  // layout without it matches the forward call's
  Layout L = carve(nullptr, N, sys->n_structs, nl->capacity, P.D, P.S, model);
  if (!ws || ws_bytes < L.bytes) return fail(NN_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.bytes);
  L = carve(ws, N, sys->n_structs, nl->capacity, P.D, P.S, model);
  hipStream_t s = (hipStream_t)stream;
  if (N == 0) return NN_OK;
  if (dL_dpos) launch_pos_grad(dL_dE, sys->atom_ptr, sys->n_structs, N, F, dL_dpos, s);
  if (dW || db) {
    const int mode = (flags & NN_BF16X3_MLP) ? 2 : (flags & NN_BF16_MLP) ? 1 : 0;
    const LaunchPlan plan = plan_for(N, nl->capacity, P, model, mode);
    launch_species_group(sys->species, N, P.S, L.sp_cnt, L.sp_off, L.scan_tmp, L.perm, L.sp_start, s);
    MlpArgs a{};
    prepare_model(model, P, L, mode != 0 && !dL_dF, a, s);
    launch_atom_weights(dL_dE, sys->atom_ptr, sys->n_structs, N, L.w_atom, s);
    if (!model_fused(model)) {
      // layer-by-layer MLP: the stashes of the energy path (deltas) or, with
      // a loss on forces, of the tangent and its reverse pass, then the sums
      a.G = L.G;
      a.perm = L.perm;
      a.sp_start = L.sp_start;
      a.E_atom = L.E_atom;
      a.lambda = L.lam;
      a.D = P.D;
      LayArgs la = lay_args(a, L);
      if (dL_dF) {
        launch_desc_tan(*sys, *nl, P, dL_dF, L.lam, plan.wpa_fwd, s);
        la.U = L.lam;
        launch_mlp_layers_tangent(la, N, s);
      } else {
        launch_mlp_layers(la, N, true, s);
      }
      LayGradOut out{};
      for (int k = 0; k < NN_MAX_SPECIES * NN_MAX_LAYERS; ++k) {
        out.dW[k] = dW ? dW[k] : nullptr;
        out.db[k] = db ? db[k] : nullptr;
      }
      launch_lay_wgrad(la, N, dL_dF != nullptr, L.partial, out, s);
      return check_launch("nn_energy_forces_grad");
    }
    WgradSrc src{};
    src.G = L.G;
    src.a1 = L.st_a1;
    src.d1 = L.st_d1;
    src.a2 = L.st_a2;
    src.d2 = L.st_d2;
    if (dL_dF) {
      // descriptor tangent along dL/dF into the lambda buffer (not needed
      // here), then the MLP with its tangent in FP32
      launch_desc_tan(*sys, *nl, P, dL_dF, L.lam, plan.wpa_fwd, s);
      MlpFmArgs f{};
      f.model = a.model;
      f.G = L.G;
      f.U = L.lam;
      f.perm = L.perm;
      f.sp_start = L.sp_start;
      f.w = L.w_atom;
      f.E_atom = L.E_atom;
      f.D = P.D;
      f.a1 = L.st_a1;
      f.t1 = L.st_t1;
      f.d1 = L.st_d1;
      f.x1 = L.st_x1;
      f.d2 = L.st_d2;
      f.x2 = L.st_x2;
      f.c3 = L.st_a2;
      launch_mlp_fm(f, model->mlp[0].width[1], model->mlp[0].width[2], N, plan.mlp_waves, s);
      src.U = L.lam;
      src.t1 = L.st_t1;
      src.x1 = L.st_x1;
      src.x2 = L.st_x2;
    } else {
      // re-run the MLP on the stored descriptors, keeping a1, a2, dE/dz1, dE/dz2
      a.G = L.G;
      a.perm = L.perm;
      a.sp_start = L.sp_start;
      a.E_atom = L.E_atom;
      a.lambda = nullptr;
      a.D = P.D;
      a.st_a1 = L.st_a1;
      a.st_d1 = L.st_d1;
      a.st_a2 = L.st_a2;
      a.st_d2 = L.st_d2;
      run_mlp(a, model, mode, N, plan.mlp_waves, s);
    }
    WgradArgs g{};
    g.perm = L.perm;
    g.sp_start = L.sp_start;
    g.w = L.w_atom;
    g.partial = L.partial;
    g.S = P.S;
    launch_wgrad(g, a.model, src, P.D, N, dW, db, s);
  }
  return check_launch("nn_energy_forces_grad");
}

nn_status nn_energy_forces_qeq(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p,
                               const nn_model* model, const nn_qeq_params* qp, const double* total_charge,
                               double* E_struct, double* charges, float* F, void* ws, size_t ws_bytes, void* stream) {
  nn_status st = check_system(sys);
  if (st) return st;
  if ((st = check_nlist(nl, sys, true))) return st;
  DescConst P;
  if ((st = make_desc_const(p, &P))) return st;
  if ((st = check_model(model, P, 3))) return st;
  if (nl->radius < p->rc) return fail(NN_E_INVALID, "list radius %g < rc %g", nl->radius, p->rc);
  const int64_t N = sys->n_atoms;
  Layout L = carve(nullptr, N, sys->n_structs, nl->capacity, P.D, P.S, model);
  if (!ws || ws_bytes < L.bytes) return fail(NN_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.bytes);
  L = carve(ws, N, sys->n_structs, nl->capacity, P.D, P.S, model);
  QeqArgs qa;
  if ((st = make_qeq_args(sys, nl, qp, P, total_charge, E_struct, charges, L, &qa))) return st;
  hipStream_t s = (hipStream_t)stream;
  if (N == 0) {
    if (sys->n_structs > 0) launch_energy_reduce(L.E_atom, sys->atom_ptr, sys->n_structs, N, E_struct, s);
    return check_launch("nn_energy_forces_qeq");
  }
  const LaunchPlan plan = plan_for(N, nl->capacity, P, model, 0);
  const bool fold_species = P.S == 1;
  if (!fold_species) {
    StageTimer t(NN_STAGE_SPECIES, s);
    launch_species_group(sys->species, N, P.S, L.sp_cnt, L.sp_off, L.scan_tmp, L.perm, L.sp_start, s);
  }
  MlpArgs a{};
  prepare_model(model, P, L, false, a, s);
  {
    StageTimer t(NN_STAGE_DESC_FWD, s);
    launch_desc_fwd(*sys, *nl, P, L.G, fold_species ? IdentityGroup{L.perm, L.sp_start} : IdentityGroup{},
                    plan.wpa_fwd, s);
  }
  a.G = L.G;
  a.perm = L.perm;
  a.sp_start = L.sp_start;
  a.E_atom = L.E_atom;
  a.lambda = L.lam;
  a.D = P.D;
  LayArgs la = lay_args(a, L);
  la.n_out = 3;
  la.out = L.qeq_out;
  la.seed = L.qeq_seed;
  {
    StageTimer t(NN_STAGE_MLP, s);
    launch_mlp_layers_outputs(la, N, s);
  }
  launch_qeq_solve(qa, s);
  if (F) {
    {
      StageTimer t(NN_STAGE_MLP, s);
      launch_mlp_layers_seeded_backward(la, N, true, s);
    }
    {
      StageTimer t(NN_STAGE_DESC_ADJ, s);
      launch_desc_adj(*sys, *nl, P, L.lam, L.pg, plan.wpa_adj, s);
    }
    StageTimer t(NN_STAGE_FORCE_GATHER, s);
    launch_force_gather(*sys, *nl, L.pg, F, EnergyJob{nullptr, sys->atom_ptr, 0, nullptr}, s);
    launch_qeq_coulomb(qa, F, s);
  }
  return check_launch("nn_energy_forces_qeq");
}

nn_status nn_energy_forces_qeq_grad(const nn_system* sys, const nn_nlist* nl, const nn_mbp_params* p,
                                    const nn_model* model, const double* dL_dE, float* const* dW, float* const* db,
                                    void* ws, size_t ws_bytes, void* stream) {
  nn_status st = check_system(sys);
  if (st) return st;
  if ((st = check_nlist(nl, sys, true))) return st;
  DescConst P;
  if ((st = make_desc_const(p, &P))) return st;
  if ((st = check_model(model, P, 3))) return st;
  if (!dL_dE && sys->n_structs > 0) return fail(NN_E_INVALID, "dL_dE is NULL");
  const int64_t N = sys->n_atoms;
  Layout L = carve(nullptr, N, sys->n_structs, nl->capacity, P.D, P.S, model);
  if (!ws || ws_bytes < L.bytes) return fail(NN_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, L.bytes);
  L = carve(ws, N, sys->n_structs, nl->capacity, P.D, P.S, model);
  hipStream_t s = (hipStream_t)stream;
  if (N == 0 || (!dW && !db)) return check_launch("nn_energy_forces_qeq_grad");
  launch_species_group(sys->species, N, P.S, L.sp_cnt, L.sp_off, L.scan_tmp, L.perm, L.sp_start, s);
  MlpArgs a{};
  prepare_model(model, P, L, false, a, s);
  launch_atom_weights(dL_dE, sys->atom_ptr, sys->n_structs, N, L.w_atom, s);
  a.G = L.G;
  a.perm = L.perm;
  a.sp_start = L.sp_start;
  a.E_atom = L.E_atom;
  a.lambda = L.lam;
  a.D = P.D;
  LayArgs la = lay_args(a, L);
  la.n_out = 3;
  la.out = L.qeq_out;
  la.seed = L.qeq_seed;
  // the stashes at the stored descriptors, then the deltas of the seeded outputs
  launch_mlp_layers_outputs(la, N, s);
  launch_mlp_layers_seeded_backward(la, N, false, s);
  LayGradOut out{};
  for (int k = 0; k < NN_MAX_SPECIES * NN_MAX_LAYERS; ++k) {
    out.dW[k] = dW ? dW[k] : nullptr;
    out.db[k] = db ? db[k] : nullptr;
  }
  launch_lay_wgrad(la, N, false, L.partial, out, s);
  return check_launch("nn_energy_forces_qeq_grad");
}

nn_status nn_md_langevin(const nn_system* sys, double* pos, double* vel, const double* inv_mass, nn_nlist* nl,
                         double rc, double skin, const nn_mbp_params* p, const nn_model* model, int32_t flags,
                         const nn_langevin* lp, const float* noise, int32_t n_steps, double* E_pot, float* F,
                         void* ws, size_t ws_bytes, void* stream) {
  nn_status st = check_system(sys);
  if (st) return st;
  if (!lp) return fail(NN_E_INVALID, "langevin parameters are NULL");
  if (!(lp->dt > 0.0) || !isfinite(lp->dt) || !(lp->friction >= 0.0) || !isfinite(lp->friction) ||
      !(lp->kT >= 0.0) || !isfinite(lp->kT))
    return fail(NN_E_INVALID, "need dt > 0, friction >= 0 and kT >= 0 (finite)");
  if (n_steps < 0) return fail(NN_E_INVALID, "n_steps < 0");
  if (flags & (NN_STORE_JACOBIAN | NN_REUSE_DESCRIPTORS))
    return fail(NN_E_INVALID, "dynamics takes only the MLP precision flags");
  const int64_t N = sys->n_atoms;
  if (N > 0 && pos != sys->pos) return fail(NN_E_INVALID, "pos must be the buffer sys->pos points at");
  if (N > 0 && (!vel || !inv_mass || !F)) return fail(NN_E_INVALID, "vel/inv_mass/F is NULL");
  if (n_steps > 0 && sys->n_structs > 0 && !E_pot) return fail(NN_E_INVALID, "E_pot is NULL");
  if (N > 0 && n_steps > 0 && lp->friction > 0.0 && !noise) return fail(NN_E_INVALID, "noise is NULL");
  if (n_steps == 0 || N == 0) return NN_OK;
  hipStream_t s = (hipStream_t)stream;
  const double c1 = exp(-lp->friction * lp->dt);
  const double c2 = sqrt(std::max(0.0, 1.0 - c1 * c1));
  const double c2_sqrt_kT = c2 * sqrt(lp->kT);
  const float* xi = lp->friction > 0.0 ? noise : nullptr;
  for (int32_t k = 0; k < n_steps; ++k) {
    launch_md_update(N, k == 0 ? kMdHalfKickDrift : kMdKickDrift, pos, vel, inv_mass, F,
                     xi ? xi + (size_t)k * 3 * (size_t)N : nullptr, lp->dt, c1, c2_sqrt_kT, s);
    if ((st = nn_build_neighbors(sys, rc, skin, nl, ws, ws_bytes, stream))) return st;
    if ((st = nn_energy_forces(sys, nl, p, model, flags, 0, E_pot + (size_t)k * sys->n_structs, nullptr, F, ws,
                               ws_bytes, stream)))
      return st;
  }
  launch_md_update(N, kMdKick, pos, vel, inv_mass, F, nullptr, lp->dt, c1, c2_sqrt_kT, s);
  return check_launch("nn_md_langevin");
}

nn_status nn_loss(const nn_system* sys, const nn_loss_params* lp, const double* E, const double* E_ref,
                  const float* F, const float* F_ref, double* L, double* dL_dE, float* dL_dF, void* ws,
                  size_t ws_bytes, void* stream) {
  nn_status st = check_system(sys);
  if (st) return st;
  if (!lp) return fail(NN_E_INVALID, "loss parameters are NULL");
  if ((lp->energy_kind != NN_LOSS_QUAD && lp->energy_kind != NN_LOSS_EXP) ||
      (lp->force_kind != NN_LOSS_QUAD && lp->force_kind != NN_LOSS_EXP))
    return fail(NN_E_INVALID, "unknown loss kind");
  if (!isfinite(lp->energy_weight) || !isfinite(lp->force_weight)) return fail(NN_E_INVALID, "weights must be finite");
  if (!L) return fail(NN_E_INVALID, "L is NULL");
  if (sys->n_structs > 0 && (!E || !E_ref || !dL_dE)) return fail(NN_E_INVALID, "E/E_ref/dL_dE is NULL");
  if ((F == nullptr) != (F_ref == nullptr)) return fail(NN_E_INVALID, "F and F_ref must both be given or both NULL");
  if (F && sys->n_atoms > 0 && !dL_dF) return fail(NN_E_INVALID, "dL_dF is NULL");
  Layout Lw = carve(nullptr, sys->n_atoms, sys->n_structs, 0, 0, 1, nullptr);
  if (!ws || ws_bytes < Lw.bytes) return fail(NN_E_WORKSPACE, "workspace %zu < %zu bytes", ws_bytes, Lw.bytes);
  Lw = carve(ws, sys->n_atoms, sys->n_structs, 0, 0, 1, nullptr);
  launch_loss(*lp, sys->atom_ptr, sys->n_structs, sys->n_atoms, E, E_ref, sys->n_atoms > 0 ? F : nullptr, F_ref, L,
              dL_dE, dL_dF, Lw.loss_partial, (hipStream_t)stream);
  return check_launch("nn_loss");
}

nn_status nn_check(const nn_nlist* nl, void* stream, int64_t* info) {
  if (!nl || !nl->meta) return fail(NN_E_INVALID, "nl/meta is NULL");
  hipStream_t s = (hipStream_t)stream;
  int64_t meta[8];
  if (hipMemcpyAsync(meta, nl->meta, sizeof meta, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(NN_E_HIP, "nn_check: %s", hipGetErrorString(hipGetLastError()));
  const int64_t err = meta[kMetaErr];
  if (info) *info = meta[kMetaNnz];
  if (err) {
    hipLaunchKernelGGL(k_zero_meta, dim3(1), dim3(1), 0, s, nl->meta + kMetaErr);  // clears error word only
    (void)hipStreamSynchronize(s);
  }
  if (err & kErrPtr) return fail(NN_E_INVALID, "atom_ptr must run from 0 to N without decreasing");
  if (err & kErrCapacity)
    return fail(NN_E_CAPACITY, "neighbor list needs %lld entries, capacity %lld", (long long)meta[kMetaNnz],
                (long long)nl->capacity);
  if (err & kErrCell) return fail(NN_E_CELL, "periodic cell narrower than 3 bins for a structure over 256 atoms");
  if (err & kErrSpecies) return fail(NN_E_DEVICE, "species index out of range");
  if (err & kErrNonFinite) return fail(NN_E_DEVICE, "non-finite position");
  if (err & kErrShift) return fail(NN_E_DEVICE, "lattice image index beyond int8");
  if (err & kErrTooMany) return fail(NN_E_DEVICE, "too many neighbors (> %d inside rc or > %d per row)", kMaxNb, kRowMax);
  if (err & kErrQeq)
    return fail(NN_E_DEVICE, "charge equilibration failed: a structure is periodic, has more than %d atoms, or its "
                             "matrix is not positive definite (its charges, energy and Coulomb forces are zero)",
                kQeqMax);
  if (err & kErrStale)
    return fail(NN_E_DEVICE, "NN_REUSE_DESCRIPTORS after a list rebuild: the stored Jacobian is stale (forces zeroed)");
  return NN_OK;
}

const char* nn_last_error(void) { return g_err; }

int64_t nn_jacobian_stride(const nn_mbp_params* p) {
  DescConst P;
  if (make_desc_const(p, &P) != NN_OK) return -1;
  return (int64_t)jacobian_floats(P.n_rad, P.S, P.n_theta, P.n_rs_ang, 1);
}

nn_status nn_timing(int32_t enable) {
  std::lock_guard<std::mutex> g(g_tmu);
  for (auto& t : g_tl) {
    (void)hipEventSynchronize(t.b);
    g_event_pool.push_back(t.a);
    g_event_pool.push_back(t.b);
  }
  g_tl.clear();
  g_timing = enable != 0;
  return NN_OK;
}

nn_status nn_timing_read(double* ms, int64_t* launches) {
  if (!ms || !launches) return fail(NN_E_INVALID, "ms/launches is NULL");
  std::lock_guard<std::mutex> g(g_tmu);
  for (int k = 0; k < NN_STAGE_COUNT; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  for (auto& t : g_tl) {
    if (hipEventSynchronize(t.b) != hipSuccess) return fail(NN_E_HIP, "nn_timing_read: event sync failed");
    float e = 0.f;
    if (hipEventElapsedTime(&e, t.a, t.b) != hipSuccess) return fail(NN_E_HIP, "nn_timing_read: elapsed failed");
    ms[t.stage] += e;
    launches[t.stage] += 1;
  }
  return NN_OK;
}

}  // extern "C"
