// Host side of libammse: validation, plans, workspace map, launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <array>
#include <vector>

#include "ammse_internal.h"

struct ammse_plan_s {
  int32_t device = 0;
  int32_t batch = 0;
  int32_t use_fast = 0;
  int32_t n_qp = 0;            // launch positions [0, n_qp): the general kernel's Q path
  ammse_options_t opt{};
  size_t ws_bytes = 0;
  ammse_desc_t* d_desc = nullptr;
  int32_t* d_cell_users = nullptr;
  // for the unrolled solver
  bool single_cell = true;     // every instance has C == 1
  bool h_disjoint = true;      // channel blocks do not overlap (dH is written)
  int64_t v_elems = 0;         // minimum length of V (complex elements)
  std::vector<std::array<int32_t, 4>> shapes;   // (U, M, N, d) per instance
  // autotuned tile shapes: host copy of the descriptors (launch order) and
  // the shape class of each launch position
  std::vector<ammse_desc_t> h_desc;
  std::vector<int8_t> tile_class;
  void* scratch = nullptr;     // this device's static workspace array (ammse_solve_noalloc)
};

namespace {

int resolved_lanczos(const ammse_options_t& o) {
  return o.lanczos_steps > 0 ? o.lanczos_steps : AMMSE_MAX_LANCZOS;
}

ammse_status_t check_options(const ammse_options_t& o) {
  if (o.precision != AMMSE_PREC_FP64 && o.precision != AMMSE_PREC_FP32 &&
      o.precision != AMMSE_PREC_BF16)
    return AMMSE_ERR_OPTION;
  if (o.max_iters < 0 || o.max_iters > 1000000) return AMMSE_ERR_OPTION;
  if (o.T_c < 0) return AMMSE_ERR_OPTION;
  if (o.warm_start != 0 && o.warm_start != 1) return AMMSE_ERR_OPTION;
  if (o.extrapolate != 0 && o.extrapolate != 1) return AMMSE_ERR_OPTION;
  if (o.rearm_at_switch != 0 && o.rearm_at_switch != 1) return AMMSE_ERR_OPTION;
  if (o.force_switch_iter != -1 && o.force_switch_iter < 1) return AMMSE_ERR_OPTION;
  if (o.lanczos_steps < 0 || o.lanczos_steps > AMMSE_MAX_LANCZOS) return AMMSE_ERR_OPTION;
  if (o.path != AMMSE_PATH_AUTO && o.path != AMMSE_PATH_GENERAL) return AMMSE_ERR_OPTION;
  if (o.refine_iters < 0) return AMMSE_ERR_OPTION;
  if (o.tile < 0 || o.tile > 3) return AMMSE_ERR_OPTION;
  if (o.step_rule != AMMSE_STEP_BOUND && o.step_rule != AMMSE_STEP_FROZEN) return AMMSE_ERR_OPTION;
  if (o.algorithm != AMMSE_ALGO_AMMMSE && o.algorithm != AMMSE_ALGO_WMMSE &&
      o.algorithm != AMMSE_ALGO_MMMSE && o.algorithm != AMMSE_ALGO_BCGD)
    return AMMSE_ERR_OPTION;
  if (o.algorithm != AMMSE_ALGO_AMMMSE && o.precision == AMMSE_PREC_BF16)
    return AMMSE_ERR_UNSUPPORTED;
  if (!(o.eps1 >= 0.0) || !(o.eps2 >= 0.0)) return AMMSE_ERR_OPTION;
  if (o.T_c == 0 && !(o.gamma_c > 0.0)) return AMMSE_ERR_OPTION;
  if (o.gamma_c != o.gamma_c) return AMMSE_ERR_OPTION;
  return AMMSE_OK;
}

}  // namespace

extern "C" {

int32_t ammse_version(void) { return AMMSE_VERSION; }

const char* ammse_status_string(ammse_status_t s) {
  switch (s) {
    case AMMSE_OK: return "success";
    case AMMSE_ERR_NULL: return "required pointer argument is NULL";
    case AMMSE_ERR_SHAPE: return "invalid instance sizes or offsets";
    case AMMSE_ERR_OPTION: return "option out of range";
    case AMMSE_ERR_WORKSPACE: return "workspace too small";
    case AMMSE_ERR_HIP: return "HIP runtime error";
    case AMMSE_ERR_UNSUPPORTED: return "outside the limits of this build";
    case AMMSE_ERR_ALLOC: return "device allocation for the plan failed";
    default: return "unknown status";
  }
}

void ammse_default_options(ammse_options_t* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->precision = AMMSE_PREC_FP32;
  opt->max_iters = 100;
  opt->T_c = 3;
  opt->warm_start = 1;
  opt->extrapolate = 1;
  opt->rearm_at_switch = 1;
  opt->force_switch_iter = -1;
  opt->lanczos_steps = 0;
  opt->path = AMMSE_PATH_AUTO;
  opt->refine_iters = 10;
  opt->algorithm = AMMSE_ALGO_AMMMSE;
  opt->tile = 0;
  opt->step_rule = AMMSE_STEP_BOUND;
  opt->eps1 = 0.1;
  opt->eps2 = 0.0;
  opt->gamma_c = 0.0;
}

ammse_status_t ammse_validate(const ammse_instance_t* table, const int32_t* cell_users,
                              int32_t batch, const ammse_options_t* opt, int64_t* h_elems,
                              int64_t* v_elems, int64_t* user_elems, int64_t* bs_elems) {
  ammse_options_t o;
  if (opt) {
    o = *opt;
  } else {
    ammse_default_options(&o);
  }
  ammse_status_t st = check_options(o);
  if (st != AMMSE_OK) return st;
  if (batch < 0) return AMMSE_ERR_SHAPE;
  if (batch > 0 && (!table || !cell_users)) return AMMSE_ERR_NULL;
  int64_t hmax = 0, vmax = 0, umax = 0, bmax = 0;
  std::vector<std::pair<int64_t, int64_t>> vspans;
  vspans.reserve(batch);
  for (int32_t i = 0; i < batch; ++i) {
    const ammse_instance_t& t = table[i];
    if (t.C < 1 || t.U < 1 || t.M < 1 || t.N < 1 || t.d < 1 || t.d > t.N) return AMMSE_ERR_SHAPE;
    if (t.cell_off < 0 || t.h_off < 0 || t.v_off < 0 || t.user_off < 0 || t.bs_off < 0)
      return AMMSE_ERR_SHAPE;
    if (t.C > AMMSE_MAX_CELLS || t.U > AMMSE_MAX_USERS || t.M > AMMSE_MAX_ANTENNAS ||
        t.N > AMMSE_MAX_RX)
      return AMMSE_ERR_UNSUPPORTED;
    int64_t su = 0;
    for (int c = 0; c < t.C; ++c) {
      const int32_t n = cell_users[(int64_t)t.cell_off + c];
      if (n < 0) return AMMSE_ERR_SHAPE;
      su += n;
    }
    if (su != t.U) return AMMSE_ERR_SHAPE;
    const int64_t hlen = (int64_t)t.C * t.U * t.N * t.M;
    const int64_t vlen = (int64_t)t.M * t.U * t.d;
    hmax = std::max(hmax, t.h_off + hlen);
    vmax = std::max(vmax, t.v_off + vlen);
    umax = std::max(umax, t.user_off + t.U);
    bmax = std::max(bmax, t.bs_off + t.C);
    vspans.emplace_back(t.v_off, vlen);
  }
  // precoder blocks are written: they must not overlap
  std::sort(vspans.begin(), vspans.end());
  for (size_t i = 1; i < vspans.size(); ++i)
    if (vspans[i - 1].first + vspans[i - 1].second > vspans[i].first) return AMMSE_ERR_SHAPE;
  if (h_elems) *h_elems = hmax;
  if (v_elems) *v_elems = vmax;
  if (user_elems) *user_elems = umax;
  if (bs_elems) *bs_elems = bmax;
  return AMMSE_OK;
}

ammse_status_t ammse_plan_create(ammse_plan_t* plan, int32_t device,
                                 const ammse_instance_t* table, const int32_t* cell_users,
                                 int32_t batch, const ammse_options_t* opt) {
  if (!plan) return AMMSE_ERR_NULL;
  ammse_options_t o;
  if (opt) {
    o = *opt;
  } else {
    ammse_default_options(&o);
  }
  ammse_status_t st =
      ammse_validate(table, cell_users, batch, &o, nullptr, nullptr, nullptr, nullptr);
  if (st != AMMSE_OK) return st;
  if (batch < 1) return AMMSE_ERR_SHAPE;
  if (hipSetDevice(device) != hipSuccess) return AMMSE_ERR_HIP;

  const int rb = (o.precision == AMMSE_PREC_FP64) ? 8 : 4;   // BF16 mode stores float
  const int ls = resolved_lanczos(o);
  // launch order: decreasing work, so the dispatcher balances uneven batches
  std::vector<int32_t> order(batch);
  std::iota(order.begin(), order.end(), 0);
  std::vector<double> cost(batch);
  for (int32_t i = 0; i < batch; ++i) {
    const ammse_instance_t& t = table[i];
    cost[i] = (double)t.C * t.U * t.N * (double)t.M * t.U * t.d;
  }
  // general kernel: the instances of its single-cell Q path first (they run in
  // their own kernel variant), each group by decreasing work
  std::vector<char> qpi(batch);
  for (int32_t i = 0; i < batch; ++i) {
    const ammse_instance_t& t = table[i];
    qpi[i] = ammse_qpath_instance(t.C, t.U, t.M, t.N, o.algorithm) ? 1 : 0;
  }
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    if (qpi[a] != qpi[b]) return qpi[a] > qpi[b];
    return cost[a] > cost[b];
  });
  int32_t n_qp = 0;
  for (int32_t i = 0; i < batch; ++i) n_qp += qpi[i];

  bool fast = (o.precision == AMMSE_PREC_FP32) && (o.path == AMMSE_PATH_AUTO) &&
              (o.algorithm == AMMSE_ALGO_AMMMSE);
  for (int32_t i = 0; fast && i < batch; ++i) {
    const ammse_instance_t& t = table[i];
    fast = ammse_fast_eligible(t.C, t.U, t.M, t.N, t.d);
  }

  std::vector<ammse_desc_t> desc(batch);
  size_t off = 0;
  int64_t ncu = 0;
  for (int32_t i = 0; i < batch; ++i) ncu = std::max<int64_t>(ncu, table[i].cell_off + table[i].C);
  for (int32_t k = 0; k < batch; ++k) {
    const ammse_instance_t& t = table[order[k]];
    ammse_desc_t& d = desc[k];
    d.C = t.C;
    d.U = t.U;
    d.M = t.M;
    d.N = t.N;
    d.d = t.d;
    d.cell_off = t.cell_off;
    d.un = t.U * t.N;
    d.ud = t.U * t.d;
    d.b = order[k];
    d.tile = 0;
    d.h_off = t.h_off;
    d.v_off = t.v_off;
    d.user_off = t.user_off;
    d.bs_off = t.bs_off;
    d.ws_off = (int64_t)off;
    if (!fast)
      off += ammse_ws_layout(rb, t.C, t.U, t.M, t.N, t.d, ls,
                             o.algorithm == AMMSE_ALGO_WMMSE || o.algorithm == AMMSE_ALGO_MMMSE,
                             o.precision == AMMSE_PREC_BF16, o.algorithm == AMMSE_ALGO_BCGD)
                 .total;
  }

  ammse_plan_s* P = new (std::nothrow) ammse_plan_s();
  if (!P) return AMMSE_ERR_ALLOC;
  {
    std::vector<std::pair<int64_t, int64_t>> hspans;
    int64_t vmax = 0;
    P->shapes.resize(batch);
    for (int32_t i = 0; i < batch; ++i) {
      const ammse_instance_t& t = table[i];
      P->single_cell = P->single_cell && t.C == 1;
      hspans.emplace_back(t.h_off, (int64_t)t.C * t.U * t.N * t.M);
      vmax = std::max(vmax, t.v_off + (int64_t)t.M * t.U * t.d);
      P->shapes[i] = {t.U, t.M, t.N, t.d};
    }
    std::sort(hspans.begin(), hspans.end());
    for (size_t i = 1; i < hspans.size(); ++i)
      if (hspans[i - 1].first + hspans[i - 1].second > hspans[i].first) P->h_disjoint = false;
    P->v_elems = vmax;
  }
  P->device = device;
  P->batch = batch;
  P->use_fast = fast ? 1 : 0;
  P->n_qp = n_qp;
  P->opt = o;
  P->opt.lanczos_steps = ls;
  // the LDS-resident kernel keeps its state on chip; its workspace holds the
  // stage-II step bound of each instance (one double per launch position)
  if (fast) off = ammse_align256(sizeof(double) * (size_t)batch);
  P->ws_bytes = std::max<size_t>(off, 256);
  P->h_desc = desc;
  P->tile_class.resize(batch);
  for (int32_t k = 0; k < batch; ++k) {
    const ammse_instance_t& t = table[order[k]];
    int32_t n = 0;
    for (int c = 0; c < t.C; ++c) n = std::max(n, cell_users[(int64_t)t.cell_off + c] * t.d);
    P->tile_class[k] = (int8_t)((n <= 16) ? 0 : (n <= 32) ? 1 : 2);
  }
  // set-up of the allocation-free solve: this device's copy of the static
  // workspace array (looked up once per device, with the device current)
  if (ammse_scratch_resolve(device, &P->scratch) != hipSuccess) {
    delete P;
    return AMMSE_ERR_HIP;
  }
  if (hipMalloc(&P->d_desc, sizeof(ammse_desc_t) * batch) != hipSuccess ||
      hipMalloc(&P->d_cell_users, sizeof(int32_t) * std::max<int64_t>(ncu, 1)) != hipSuccess) {
    if (P->d_desc) (void)hipFree(P->d_desc);
    delete P;
    return AMMSE_ERR_ALLOC;
  }
  if (hipMemcpy(P->d_desc, desc.data(), sizeof(ammse_desc_t) * batch, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(P->d_cell_users, cell_users, sizeof(int32_t) * ncu, hipMemcpyHostToDevice) !=
          hipSuccess) {
    (void)hipFree(P->d_desc);
    (void)hipFree(P->d_cell_users);
    delete P;
    return AMMSE_ERR_HIP;
  }
  *plan = P;
  return AMMSE_OK;
}

ammse_status_t ammse_plan_workspace_size(ammse_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return AMMSE_ERR_NULL;
  *bytes = plan->ws_bytes;
  return AMMSE_OK;
}

ammse_status_t ammse_plan_info(ammse_plan_t plan, int32_t* kernel, size_t* lds_bytes) {
  if (!plan) return AMMSE_ERR_NULL;
  if (kernel) *kernel = plan->use_fast ? AMMSE_KERNEL_LDS_MFMA : AMMSE_KERNEL_GENERAL;
  if (lds_bytes) *lds_bytes = plan->use_fast ? ammse_fast_lds_bytes() : ammse_general_lds_bytes(plan->opt.precision, plan->opt.algorithm);
  return AMMSE_OK;
}

ammse_status_t ammse_plan_destroy(ammse_plan_t plan) {
  if (!plan) return AMMSE_OK;
  (void)hipSetDevice(plan->device);
  (void)hipFree(plan->d_desc);
  (void)hipFree(plan->d_cell_users);
  delete plan;
  return AMMSE_OK;
}

static ammse_status_t launch(ammse_plan_t plan, ammse_kparams_t& k, hipStream_t stream) {
  if (hipSetDevice(plan->device) != hipSuccess) return AMMSE_ERR_HIP;
  hipError_t e = plan->use_fast ? ammse_launch_fast_fp32(k, stream)
                 : (plan->opt.precision == AMMSE_PREC_FP64) ? ammse_launch_fp64(k, stream)
                                                            : ammse_launch_fp32(k, stream);
  return (e == hipSuccess) ? AMMSE_OK : AMMSE_ERR_HIP;
}

static void fill_common(ammse_plan_t plan, ammse_kparams_t& k) {
  std::memset(&k, 0, sizeof(k));
  const ammse_options_t& o = plan->opt;
  k.desc = plan->d_desc;
  k.cell_users = plan->d_cell_users;
  k.batch = plan->batch;
  k.n_qp = plan->n_qp;
  k.max_iters = o.max_iters;
  k.T_c = o.T_c;
  k.warm_start = o.warm_start;
  k.extrapolate = o.extrapolate;
  k.rearm = o.rearm_at_switch;
  k.force_switch_iter = o.force_switch_iter;
  k.lanczos_steps = o.lanczos_steps;
  k.trace_len = o.max_iters + 1;
  k.eps1 = o.eps1;
  k.eps2 = o.eps2;
  k.gamma_c = o.gamma_c;
  k.lowp_iters = (o.precision == AMMSE_PREC_BF16) ? std::max(0, o.max_iters - o.refine_iters) : -1;
  k.algorithm = o.algorithm;
  k.bf16_copies = o.precision == AMMSE_PREC_BF16;
  k.tile_force = o.tile;
  k.step_rule = o.step_rule;
}

ammse_status_t ammse_solve(ammse_plan_t plan, const void* H, const double* sigma2,
                           const double* alpha, const double* P, void* V, double* wsr,
                           int32_t* iters, int32_t* switch_iter, int32_t* status,
                           double* wsr_trace, const int32_t* force_switch, void* workspace,
                           size_t workspace_bytes, ammse_stream_t stream) {
  if (!plan || !H || !sigma2 || !alpha || !P || !V || !wsr || !workspace) return AMMSE_ERR_NULL;
  if (workspace_bytes < plan->ws_bytes) return AMMSE_ERR_WORKSPACE;
  if (((uintptr_t)workspace & 255) != 0) return AMMSE_ERR_WORKSPACE;
  ammse_kparams_t k;
  fill_common(plan, k);
  k.H = H;
  k.sigma2 = sigma2;
  k.alpha = alpha;
  k.P = P;
  k.V = V;
  k.wsr = wsr;
  k.iters = iters;
  k.switch_iter = switch_iter;
  k.status = status;
  k.trace = wsr_trace;
  k.force_switch = force_switch;
  k.ws = (char*)workspace;
  k.wsr_only = 0;
  return launch(plan, k, (hipStream_t)stream);
}

ammse_status_t ammse_solve_noalloc(ammse_plan_t plan, const void* H, const double* sigma2,
                                   const double* alpha, const double* P, void* V, double* wsr,
                                   int32_t* iters, int32_t* switch_iter, int32_t* status,
                                   double* wsr_trace, const int32_t* force_switch,
                                   ammse_stream_t stream) {
  if (!plan) return AMMSE_ERR_NULL;
  if (plan->ws_bytes > AMMSE_SCRATCH_BYTES) return AMMSE_ERR_WORKSPACE;
  if (!plan->scratch) return AMMSE_ERR_HIP;
  return ammse_solve(plan, H, sigma2, alpha, P, V, wsr, iters, switch_iter, status, wsr_trace,
                     force_switch, plan->scratch, AMMSE_SCRATCH_BYTES, stream);
}

ammse_status_t ammse_wsr(ammse_plan_t plan, const void* H, const double* sigma2,
                         const double* alpha, const void* V, double* wsr, void* workspace,
                         size_t workspace_bytes, ammse_stream_t stream) {
  if (!plan || !H || !sigma2 || !alpha || !V || !wsr || !workspace) return AMMSE_ERR_NULL;
  if (workspace_bytes < plan->ws_bytes) return AMMSE_ERR_WORKSPACE;
  if (((uintptr_t)workspace & 255) != 0) return AMMSE_ERR_WORKSPACE;
  ammse_kparams_t k;
  fill_common(plan, k);
  k.H = H;
  k.sigma2 = sigma2;
  k.alpha = alpha;
  k.P = nullptr;   // budgets are not read when only the WSR is evaluated
  k.V = const_cast<void*>(V);
  k.wsr = wsr;
  k.ws = (char*)workspace;
  k.wsr_only = 1;
  k.max_iters = 0;
  k.trace_len = 1;
  k.lowp_iters = -1;   // the WSR of V is evaluated with float products
  return launch(plan, k, (hipStream_t)stream);
}

ammse_status_t ammse_autotune(ammse_plan_t plan, const void* H, const double* sigma2,
                              const double* alpha, const double* P, const void* V,
                              void* workspace, size_t workspace_bytes, int32_t* choice,
                              ammse_stream_t stream) {
  if (choice)
    for (int c = 0; c < 3; ++c) choice[c] = -1;
  if (!plan || !H || !sigma2 || !alpha || !P || !V || !workspace) return AMMSE_ERR_NULL;
  if (workspace_bytes < plan->ws_bytes) return AMMSE_ERR_WORKSPACE;
  if (((uintptr_t)workspace & 255) != 0) return AMMSE_ERR_WORKSPACE;
  if (plan->use_fast || plan->opt.precision == AMMSE_PREC_FP64) return AMMSE_OK;
  if (hipSetDevice(plan->device) != hipSuccess) return AMMSE_ERR_HIP;
  hipStream_t s = (hipStream_t)stream;
  const size_t vbytes = (size_t)plan->v_elems * 2 * sizeof(float);
  const int32_t nsample_max = 64;
  void* Vs = nullptr;
  double* wsr = nullptr;
  ammse_desc_t* dd = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ammse_status_t st = AMMSE_OK;
  auto cleanup = [&]() {
    if (Vs) (void)hipFree(Vs);
    if (wsr) (void)hipFree(wsr);
    if (dd) (void)hipFree(dd);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc(&Vs, std::max<size_t>(vbytes, 16)) != hipSuccess ||
      hipMalloc((void**)&wsr, sizeof(double) * plan->batch) != hipSuccess ||
      hipMalloc((void**)&dd, sizeof(ammse_desc_t) * nsample_max) != hipSuccess) {
    cleanup();
    return AMMSE_ERR_ALLOC;
  }
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return AMMSE_ERR_HIP;
  }
  int32_t picked[3] = {-1, -1, -1};
  for (int cls = 0; cls < 3 && st == AMMSE_OK; ++cls) {
    std::vector<int32_t> pos;
    for (int32_t k = 0; k < plan->batch; ++k)
      if (plan->tile_class[k] == cls) pos.push_back(k);
    if (pos.empty()) continue;
    // evenly spaced sample of the class (launch order is by decreasing work)
    std::vector<ammse_desc_t> sample;
    const size_t ns = std::min<size_t>(pos.size(), nsample_max);
    for (size_t q = 0; q < ns; ++q) sample.push_back(plan->h_desc[pos[q * pos.size() / ns]]);
    // Q-path instances first, as in the plan's launch order
    std::stable_partition(sample.begin(), sample.end(), [&](const ammse_desc_t& d) {
      return ammse_qpath_instance(d.C, d.U, d.M, d.N, plan->opt.algorithm);
    });
    int32_t sample_qp = 0;
    for (const auto& d : sample)
      sample_qp += ammse_qpath_instance(d.C, d.U, d.M, d.N, plan->opt.algorithm) ? 1 : 0;
    float best_ms = 0.f;
    for (int v = 0; v < AMMSE_TILE_SHAPES && st == AMMSE_OK; ++v) {
      for (auto& d : sample) d.tile = v;
      if (hipMemcpyAsync(dd, sample.data(), sizeof(ammse_desc_t) * ns, hipMemcpyHostToDevice, s) !=
          hipSuccess) {
        st = AMMSE_ERR_HIP;
        break;
      }
      ammse_kparams_t k;
      fill_common(plan, k);
      k.desc = dd;
      k.batch = (int32_t)ns;
      k.n_qp = sample_qp;
      k.max_iters = std::min(plan->opt.max_iters, 8);
      k.trace_len = k.max_iters + 1;
      if (k.lowp_iters >= 0) k.lowp_iters = std::max(0, k.max_iters - std::min(plan->opt.refine_iters, 2));
      k.tile_force = 0;
      k.H = H;
      k.sigma2 = sigma2;
      k.alpha = alpha;
      k.P = P;
      k.V = Vs;
      k.wsr = wsr;
      k.ws = (char*)workspace;
      float ms = 0.f;
      for (int rep = 0; rep < 3 && st == AMMSE_OK; ++rep) {   // one warm-up, two timed
        if (hipMemcpyAsync(Vs, V, vbytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipEventRecord(e0, s) != hipSuccess) {
          st = AMMSE_ERR_HIP;
          break;
        }
        st = launch(plan, k, s);
        if (st != AMMSE_OK) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          st = AMMSE_ERR_HIP;
          break;
        }
        float t = 0.f;
        if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
          st = AMMSE_ERR_HIP;
          break;
        }
        if (rep == 1 || (rep == 2 && t < ms)) ms = t;
      }
      if (st == AMMSE_OK && (picked[cls] < 0 || ms < best_ms)) {
        picked[cls] = v;
        best_ms = ms;
      }
    }
    if (st == AMMSE_OK)
      for (int32_t k : pos) plan->h_desc[k].tile = picked[cls];
  }
  if (st == AMMSE_OK &&
      hipMemcpy(plan->d_desc, plan->h_desc.data(), sizeof(ammse_desc_t) * plan->batch,
                hipMemcpyHostToDevice) != hipSuccess)
    st = AMMSE_ERR_HIP;
  cleanup();
  if (st == AMMSE_OK && choice)
    for (int c = 0; c < 3; ++c) choice[c] = picked[c];
  return st;
}

static ammse_status_t unroll_check(ammse_plan_t plan, int32_t ckpt_every) {
  if (!plan) return AMMSE_ERR_NULL;
  if (ckpt_every < 1) return AMMSE_ERR_OPTION;
  if (!plan->single_cell || plan->opt.algorithm != AMMSE_ALGO_AMMMSE ||
      plan->opt.precision == AMMSE_PREC_BF16)
    return AMMSE_ERR_UNSUPPORTED;
  return AMMSE_OK;
}

static size_t unroll_stride(ammse_plan_t plan, int32_t K) {
  const int rb = (plan->opt.precision == AMMSE_PREC_FP64) ? 8 : 4;
  size_t m = 256;
  for (const auto& s : plan->shapes)
    m = std::max(m, ammse_unroll_layout(rb, s[0], s[1], s[2], s[3], K).total);
  return m;
}

ammse_status_t ammse_unrolled_workspace_size(ammse_plan_t plan, int32_t ckpt_every,
                                             size_t* ws_bytes, size_t* ckpt_bytes) {
  const ammse_status_t st = unroll_check(plan, ckpt_every);
  if (st != AMMSE_OK) return st;
  if (!ws_bytes || !ckpt_bytes) return AMMSE_ERR_NULL;
  const int rb = (plan->opt.precision == AMMSE_PREC_FP64) ? 8 : 4;
  const int64_t T = plan->opt.max_iters;
  const int64_t nck = std::max<int64_t>(1, (T + ckpt_every - 1) / ckpt_every);
  *ws_bytes = unroll_stride(plan, ckpt_every) * (size_t)plan->batch;
  *ckpt_bytes = (size_t)(2 * nck * plan->v_elems) * 2 * rb;
  return AMMSE_OK;
}

static void fill_unroll(ammse_plan_t plan, int32_t K, ammse_unroll_params_t& q) {
  std::memset(&q, 0, sizeof(q));
  const int64_t T = plan->opt.max_iters;
  q.ckpt_every = K;
  q.nck = (int32_t)std::max<int64_t>(1, (T + K - 1) / K);
  q.ws_stride = unroll_stride(plan, K);
  q.fp64 = plan->opt.precision == AMMSE_PREC_FP64;
}

ammse_status_t ammse_unrolled_forward(ammse_plan_t plan, const void* H, const double* sigma2,
                                      const double* alpha, const double* P, void* V,
                                      const double* gamma, int32_t ckpt_every, double* wsr,
                                      int32_t* switch_iter, int32_t* status, double* wsr_trace,
                                      const int32_t* force_switch, void* ckpt, void* workspace,
                                      size_t workspace_bytes, ammse_stream_t stream) {
  const ammse_status_t st = unroll_check(plan, ckpt_every);
  if (st != AMMSE_OK) return st;
  if (!H || !sigma2 || !alpha || !P || !V || !gamma || !wsr || !switch_iter || !ckpt ||
      !workspace)
    return AMMSE_ERR_NULL;
  size_t need = 0, cneed = 0;
  (void)ammse_unrolled_workspace_size(plan, ckpt_every, &need, &cneed);
  if (workspace_bytes < need || ((uintptr_t)workspace & 255) != 0) return AMMSE_ERR_WORKSPACE;
  ammse_kparams_t k;
  fill_common(plan, k);
  k.H = H;
  k.sigma2 = sigma2;
  k.alpha = alpha;
  k.P = P;
  k.V = V;
  k.wsr = wsr;
  k.switch_iter = switch_iter;
  k.status = status;
  k.trace = wsr_trace;
  k.force_switch = force_switch;
  k.ws = (char*)workspace;
  ammse_unroll_params_t q;
  fill_unroll(plan, ckpt_every, q);
  q.gamma = gamma;
  q.ckpt = ckpt;
  if (hipSetDevice(plan->device) != hipSuccess) return AMMSE_ERR_HIP;
  return ammse_launch_unroll(k, q, false, (hipStream_t)stream) == hipSuccess ? AMMSE_OK
                                                                               : AMMSE_ERR_HIP;
}

ammse_status_t ammse_unrolled_backward(ammse_plan_t plan, const void* H, const double* sigma2,
                                       const double* alpha, const double* P, const double* gamma,
                                       int32_t ckpt_every, const int32_t* switch_iter,
                                       const void* ckpt, const double* dwsr, void* dH,
                                       double* dgamma, void* workspace, size_t workspace_bytes,
                                       ammse_stream_t stream) {
  const ammse_status_t st = unroll_check(plan, ckpt_every);
  if (st != AMMSE_OK) return st;
  if (!H || !sigma2 || !alpha || !P || !gamma || !switch_iter || !ckpt || !dwsr || !dH ||
      !dgamma || !workspace)
    return AMMSE_ERR_NULL;
  if (!plan->h_disjoint) return AMMSE_ERR_SHAPE;
  size_t need = 0, cneed = 0;
  (void)ammse_unrolled_workspace_size(plan, ckpt_every, &need, &cneed);
  if (workspace_bytes < need || ((uintptr_t)workspace & 255) != 0) return AMMSE_ERR_WORKSPACE;
  ammse_kparams_t k;
  fill_common(plan, k);
  k.H = H;
  k.sigma2 = sigma2;
  k.alpha = alpha;
  k.P = P;
  k.ws = (char*)workspace;
  ammse_unroll_params_t q;
  fill_unroll(plan, ckpt_every, q);
  q.gamma = gamma;
  q.ckpt = const_cast<void*>(ckpt);
  q.dH = dH;
  q.dgamma = dgamma;
  q.switch_iter = switch_iter;
  q.dwsr = dwsr;
  if (hipSetDevice(plan->device) != hipSuccess) return AMMSE_ERR_HIP;
  return ammse_launch_unroll(k, q, true, (hipStream_t)stream) == hipSuccess ? AMMSE_OK
                                                                              : AMMSE_ERR_HIP;
}

}  // extern "C"
