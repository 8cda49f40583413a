// Host side of libsgq: argument validation, plans (node order, workspace), the C ABI.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "sgq.h"
#include "sgq_common.h"
#include "tridiag.h"

namespace sgq {
hipError_t launch_forward(const LaunchParams& P, bool fp64, int grid, int block, int kg,
                          hipStream_t s);
hipError_t launch_setup(const LaunchParams& P, bool fp64, const double* v64, void* vstore,
                        void* chi, int32_t* g0, double* vmax, hipStream_t s);
hipError_t launch_weighted_sum(const double* e, const double* w, int n, double* out,
                               hipStream_t s);
hipError_t launch_gauss_rule(const LaunchParams& P, hipStream_t s);
hipError_t launch_cluster_energy(const double* e_node, int nq, const int64_t* offset,
                                 const int32_t* member, int64_t n_members, int n_esp,
                                 const double* esp_weight, double* fbar, double* energy,
                                 int* status, hipStream_t s);
hipError_t launch_fermi_level(const double* tw, const double* weight, int nq, int kmax,
                              double ne, double kT, double tol, double* out, int* status,
                              double* ws, hipStream_t s);
hipError_t launch_backward(const LaunchParams& P, bool fp64, int grid, int block, int kg,
                           hipStream_t s);
bool backward_wide_node(int half_width);
hipError_t launch_queue_reset(int* queue, hipStream_t s);
hipError_t launch_tbar(const LaunchParams& P, int grid, double* zscratch, size_t zstride,
                       double* tbar, int32_t* tbar_k, hipStream_t s);
hipError_t launch_backward_gather(const LaunchParams& P, bool fp64, const int32_t* cell_start,
                                  const int32_t* cell_nodes, int ncells, double* dV, double* dR,
                                  double* dE, hipStream_t s);
hipError_t launch_zero(double* p, size_t n, hipStream_t s);
hipError_t launch_plain(const LaunchParams& P, bool fp64, const int32_t* h_center,
                        const int32_t* h_hw, const int32_t* h_depth, void* scratch, hipStream_t s);
size_t plain_scratch_bytes(size_t npad, int kmax, bool fp64);
int backward_max_depth();
size_t backward_slot_doubles();
int gather_cell();
hipError_t launch_vloc_backward(const double* dV, const double* R, int M, int nx, int ny, int nz,
                                double h, double depth, double sigma, double cutoff, double* dR,
                                hipStream_t s);
}  // namespace sgq

using namespace sgq;

static int fail(int code, const std::string& msg) { return report_error(code, msg); }

#define HIP_OR_FAIL(expr)                                                             \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return fail(SGQ_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// One captured launch sequence of a compute call and the arguments it was captured with.
struct GraphCache {
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;
  std::vector<uint64_t> key;
};

struct sgq_plan {
  sgq_problem prob{};
  int device = 0;
  int kmax = 0, box_m = 0, kg = 8, block = 256, grid = 0;
  int slots = 0;            // Lanczos workspace slots allocated (>= grid)
  double norm_s = 0, norm_p = 0;
  size_t npad = 0, slot_stride = 0, n_grid = 0;
  bool fp64 = false;
  std::vector<int32_t> h_center, h_hw, h_depth, h_order;
  int32_t *d_order = nullptr, *d_center = nullptr, *d_hw = nullptr, *d_depth = nullptr;
  void *d_W = nullptr, *d_U = nullptr, *d_v = nullptr, *d_chi = nullptr;
  int32_t* d_g0 = nullptr;
  double* d_vmax = nullptr;
  int* d_queue = nullptr;
  int* d_status = nullptr;
  double* d_enode = nullptr;
  double* d_tri = nullptr;
  int32_t* d_trik = nullptr;
  double* d_fermi = nullptr;   // Fermi-level state and per-workgroup partial sums
  unsigned long long* d_hash = nullptr;   // input hashes: last forward call, current backward
  // retained forward bases (sgq_plan_set_retain): valid after a forward call with these
  // input pointers, consumed by the next backward call
  bool retain = false, ret_valid = false;
  const void* ret_key[3] = {nullptr, nullptr, nullptr};
  // the last forward launch covered every node with these inputs, so the tridiagonals it
  // stored serve the backward's eigensolve pre-pass
  bool tri_valid = false;
  const void* tri_key[3] = {nullptr, nullptr, nullptr};
  void* d_Wr = nullptr;
  void* d_Ur = nullptr;
  int32_t* d_ret_slot = nullptr;   // [Nq] place of each node in the retained storage, or -1
  int64_t ret_nodes = 0;
  // backward state (allocated on the first backward call)
  bool bwd_ready = false;
  int grid_bwd = 0;
  // the backward's node queue: the FP32 nodes of the 512-lane launch first (n_bwide), then
  // the others, each part in cost order
  int32_t* d_border = nullptr;
  int n_bwide = 0;
  size_t bwd_slot_stride = 0;
  void* d_Wb = nullptr;
  double* d_Zb = nullptr;
  double* d_tbar = nullptr;      // pre-pass alphabar / betabar per node
  int32_t* d_tbar_k = nullptr;
  double* d_zpre = nullptr;      // pre-pass eigenvector scratch per workgroup
  size_t zpre_stride = 0;
  int grid_pre = 0;
  void* d_P = nullptr;
  int64_t* d_cube_off = nullptr;
  double* d_dRp = nullptr;
  double* d_dEp = nullptr;
  int32_t* d_node_atoms = nullptr;
  int32_t* d_cell_start = nullptr;
  int32_t* d_cell_nodes = nullptr;
  int ncells = 0;
  int ncu = 0;
  int schedule = SGQ_SCHEDULE_BATCHED;
  void* d_plain = nullptr;
  hipStream_t last = nullptr;
  std::vector<void*> allocs;
  bool use_graph = true;
  GraphCache graphs[2];     // rho_quadrature, band_energy
  bool tuned = false;
};

static void free_all(sgq_plan* p) {
  for (GraphCache& g : p->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    g.key.clear();
  }
  for (void* a : p->allocs) (void)hipFree(a);
  p->allocs.clear();
}

template <typename T>
static hipError_t dalloc(sgq_plan* p, T** out, size_t bytes) {
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, bytes ? bytes : 16);
  if (e == hipSuccess) {
    p->allocs.push_back(ptr);
    *out = reinterpret_cast<T*>(ptr);
  }
  return e;
}

// Continuum normalisation of the projectors: int chi^2 d^3r = 1 (composite Simpson).
static void projector_norms(double rg, double rc, double* ns, double* np_) {
  const int n = 200000;
  const double dr = rc / n;
  double is = 0.0, ip = 0.0;
  for (int i = 0; i <= n; ++i) {
    double r = i * dr;
    double t = 1.0 - (r * r) / (rc * rc);
    double g = std::exp(-r * r / (2.0 * rg * rg)) * t * t * t;
    double fs = 4.0 * M_PI * r * r * g * g;
    double fp = fs * r * r / (3.0 * rg * rg);
    double wgt = (i == 0 || i == n) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
    is += wgt * fs;
    ip += wgt * fp;
  }
  is *= dr / 3.0;
  ip *= dr / 3.0;
  *ns = 1.0 / std::sqrt(is);
  *np_ = 1.0 / std::sqrt(ip);
}

extern "C" int sgq_plan_create(const sgq_problem* prob, const int64_t* center,
                               const int32_t* half_width, const int32_t* depth, sgq_plan** out) {
  if (!out) return fail(SGQ_EINVAL, "out is null");
  *out = nullptr;
  int st = sgq_validate(prob, center, half_width, depth);
  if (st != SGQ_OK) return st;
  sgq_plan* p = new sgq_plan();
  p->prob = *prob;
  p->fp64 = prob->precision == SGQ_FP64;
  HIP_OR_FAIL(hipGetDevice(&p->device));
  int ncu = 0;
  HIP_OR_FAIL(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, p->device));
  p->ncu = ncu;
  const int nq = prob->n_nodes;
  p->n_grid = (size_t)prob->n[0] * prob->n[1] * prob->n[2];
  p->box_m = prob->n_proj ? box_half_width(prob->proj_rc, prob->h) : 0;
  if (prob->n_proj) projector_norms(prob->proj_rg, prob->proj_rc, &p->norm_s, &p->norm_p);
  p->h_center.resize(nq);
  p->h_hw.assign(half_width, half_width + nq);
  p->h_depth.assign(depth, depth + nq);
  size_t nmax = 1;
  std::vector<double> cost(nq);
  for (int q = 0; q < nq; ++q) {
    p->h_center[q] = (int32_t)center[q];
    size_t n = half_width[q] < 0 ? p->n_grid : (size_t)std::pow(2 * half_width[q] + 1, 3);
    nmax = std::max(nmax, n);
    p->kmax = std::max(p->kmax, (int)depth[q]);
    double K = depth[q];
    cost[q] = (double)n * (3.0 * K + K * (K + 1.0) / 2.0);
  }
  if (p->kmax == 0) p->kmax = 1;
  p->h_order.resize(nq);
  std::iota(p->h_order.begin(), p->h_order.end(), 0);
  std::stable_sort(p->h_order.begin(), p->h_order.end(),
                   [&](int a, int b) { return cost[a] > cost[b]; });
  // basis vectors spanned by one lane group in the fused sweep
  int kg_need = (p->kmax + 3) / 4;
  p->kg = kg_need <= 8 ? 8 : (kg_need <= 16 ? 16 : 32);
  p->block = 256;
  int wg_per_cu = 2;
  if (const char* env = std::getenv("SGQ_WG_PER_CU")) wg_per_cu = std::max(1, atoi(env));
  if (const char* env = std::getenv("SGQ_BLOCK")) {
    int b = atoi(env);
    p->block = (b == 128 || b == 512) && !p->fp64 ? b : 256;
  }
  p->grid = std::max(1, std::min(nq, ncu * wg_per_cu));
  p->slots = p->grid;
  p->npad = (nmax + 63) / 64 * 64;
  p->slot_stride = (size_t)p->kmax * p->npad;
  const size_t es = p->fp64 ? 8 : 4;
  // the sweep addresses a node's basis with 32-bit byte offsets
  if (p->slot_stride * es >= ((size_t)1 << 31)) {
    delete p;
    return fail(SGQ_EINVAL, "a node's Lanczos basis (depth x cube points) exceeds 2 GiB");
  }
  hipError_t e = hipSuccess;
  e = e ? e : dalloc(p, &p->d_order, nq * 4);
  e = e ? e : dalloc(p, &p->d_center, nq * 4);
  e = e ? e : dalloc(p, &p->d_hw, nq * 4);
  e = e ? e : dalloc(p, &p->d_depth, nq * 4);
  e = e ? e : dalloc(p, &p->d_W, (size_t)p->slots * p->slot_stride * es);
  e = e ? e : dalloc(p, &p->d_U, (size_t)p->slots * p->npad * es);
  if (!p->fp64) e = e ? e : dalloc(p, &p->d_v, p->n_grid * es);
  int B = 2 * p->box_m + 1;
  if (prob->n_proj) {
    e = e ? e : dalloc(p, &p->d_chi, (size_t)std::max(1, prob->n_atoms) * B * B * B * 4 * es);
    e = e ? e : dalloc(p, &p->d_g0, (size_t)std::max(1, prob->n_atoms) * 3 * 4);
  }
  e = e ? e : dalloc(p, &p->d_vmax, 8);
  e = e ? e : dalloc(p, &p->d_queue, 8);
  e = e ? e : dalloc(p, &p->d_status, 8);
  e = e ? e : dalloc(p, &p->d_enode, (size_t)nq * 8);
  e = e ? e : dalloc(p, &p->d_tri, (size_t)nq * 2 * p->kmax * 8);
  e = e ? e : dalloc(p, &p->d_trik, (size_t)nq * 4);
  e = e ? e : dalloc(p, &p->d_fermi, (size_t)(16 + 4 * kFermiBlocks) * 8);
  e = e ? e : dalloc(p, &p->d_hash, 2 * sizeof(unsigned long long));
  if (e != hipSuccess) {
    free_all(p);
    delete p;
    (void)hipGetLastError();
    return fail(SGQ_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
  }
  e = hipMemcpy(p->d_order, p->h_order.data(), nq * 4, hipMemcpyHostToDevice);
  e = e ? e : hipMemcpy(p->d_center, p->h_center.data(), nq * 4, hipMemcpyHostToDevice);
  e = e ? e : hipMemcpy(p->d_hw, p->h_hw.data(), nq * 4, hipMemcpyHostToDevice);
  e = e ? e : hipMemcpy(p->d_depth, p->h_depth.data(), nq * 4, hipMemcpyHostToDevice);
  e = e ? e : hipMemset(p->d_status, 0, 8);
  e = e ? e : hipMemset(p->d_hash, 0, 2 * sizeof(unsigned long long));
  if (e != hipSuccess) {
    free_all(p);
    delete p;
    return fail(SGQ_EHIP, std::string("plan upload failed: ") + hipGetErrorString(e));
  }
  *out = p;
  return SGQ_OK;
}

extern "C" int sgq_plan_destroy(sgq_plan* plan) {
  if (!plan) return SGQ_OK;
  (void)hipSetDevice(plan->device);
  if (plan->last) (void)hipStreamSynchronize(plan->last);
  (void)hipDeviceSynchronize();
  free_all(plan);
  delete plan;
  return SGQ_OK;
}

static int check_call(sgq_plan* plan, const double* v_loc, const double* atom_R,
                      const double* proj_E, double mu, double kT) {
  if (!plan) return fail(SGQ_EINVAL, "plan is null");
  if (!v_loc) return fail(SGQ_EINVAL, "v_loc is null");
  if (!(kT > 0.0) || !std::isfinite(kT)) return fail(SGQ_EINVAL, "kT must be finite and > 0");
  if (!std::isfinite(mu)) return fail(SGQ_EINVAL, "mu must be finite");
  if (plan->prob.n_proj && plan->prob.n_atoms > 0 && (!atom_R || !proj_E))
    return fail(SGQ_EINVAL, "atom_R and proj_E are required when projectors are planned");
  return SGQ_OK;
}

static LaunchParams base_params(sgq_plan* p, const double* v_loc, const double* atom_R,
                                const double* proj_E, double mu, double kT) {
  LaunchParams P{};
  P.nx = p->prob.n[0];
  P.ny = p->prob.n[1];
  P.nz = p->prob.n[2];
  P.h = p->prob.h;
  P.n_atoms = p->prob.n_atoms;
  P.n_proj = p->prob.n_proj;
  P.box_m = p->box_m;
  P.proj_norm_s = p->norm_s;
  P.proj_norm_p = p->norm_p;
  P.proj_rg = p->prob.proj_rg;
  P.proj_rc = p->prob.proj_rc;
  P.n_nodes = p->prob.n_nodes;
  P.order = p->d_order;
  P.center = p->d_center;
  P.half_width = p->d_hw;
  P.depth = p->d_depth;
  P.v = p->fp64 ? (const void*)v_loc : (const void*)p->d_v;
  P.atom_R = atom_R;
  P.proj_E = proj_E;
  P.chi = p->d_chi;
  P.atom_g0 = p->d_g0;
  P.vmax = p->d_vmax;
  P.mu = mu;
  P.kT = kT;
  P.tau = p->fp64 ? 1e-12 : 1e-6;
  P.W = p->d_W;
  P.U = p->d_U;
  P.npad = p->npad;
  P.slot_stride = p->slot_stride;
  P.wbs = p->kmax * 64;
  P.queue = p->d_queue;
  P.status = p->d_status;
  P.kmax_out = p->kmax;
  P.tri = p->d_tri;
  P.tri_k = p->d_trik;
  P.Wr = p->retain ? p->d_Wr : nullptr;
  P.Ur = p->retain ? p->d_Ur : nullptr;
  P.ret_slot = p->retain ? p->d_ret_slot : nullptr;
  P.hash = p->d_hash;
  P.hash_slot = 0;
  return P;
}

// The launches of one forward call: potential copy and projector offsets, the persistent
// Lanczos-Gauss kernel and, for the energy, the node-weighted sum.
static hipError_t forward_sequence(sgq_plan* p, const LaunchParams& P, const double* v_loc,
                                   const double* node_weight, double* omega, hipStream_t s) {
  hipError_t e = launch_setup(P, p->fp64, v_loc, p->d_v, p->d_chi, p->d_g0, p->d_vmax, s);
  if (e == hipSuccess && p->prob.n_nodes > 0)
    e = launch_forward(P, p->fp64, p->grid, p->block, p->kg, s);
  if (e == hipSuccess) e = launch_gauss_rule(P, s);
  if (e == hipSuccess && omega)
    e = launch_weighted_sum(P.e_node, node_weight, p->prob.n_nodes, omega, s);
  return e;
}

// Runs the forward sequence on stream s.  On a stream that is not the legacy default
// stream and not already being captured, the sequence is captured once into a HIP graph
// and replayed while the call arguments (pointers, scalars, launch shape) are unchanged;
// a changed argument re-captures it.  The sequence holds kernels only (no memset nodes).
// After a forward launch with retention on, the retained bases belong to these inputs.
static void mark_retained(sgq_plan* p, const double* v_loc, const LaunchParams& P) {
  p->ret_valid = p->retain;
  p->ret_key[0] = v_loc;
  p->ret_key[1] = P.atom_R;
  p->ret_key[2] = P.proj_E;
  p->tri_valid = true;
  p->tri_key[0] = v_loc;
  p->tri_key[1] = P.atom_R;
  p->tri_key[2] = P.proj_E;
}

static int run_forward(sgq_plan* p, int kind, LaunchParams& P, const double* v_loc,
                       const double* node_weight, double* omega, hipStream_t s) {
  p->ret_valid = false;
  p->tri_valid = false;
  HIP_OR_FAIL(hipSetDevice(p->device));
  p->last = s;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (s) HIP_OR_FAIL(hipStreamIsCapturing(s, &cap));
  if (!p->use_graph || !s || cap != hipStreamCaptureStatusNone) {
    HIP_OR_FAIL(forward_sequence(p, P, v_loc, node_weight, omega, s));
    mark_retained(p, v_loc, P);
    return SGQ_OK;
  }
  auto bits = [](double d) { uint64_t u; std::memcpy(&u, &d, 8); return u; };
  std::vector<uint64_t> key = {
      (uint64_t)(uintptr_t)s, (uint64_t)(uintptr_t)v_loc, (uint64_t)(uintptr_t)P.atom_R,
      (uint64_t)(uintptr_t)P.proj_E, (uint64_t)(uintptr_t)P.rho, (uint64_t)(uintptr_t)P.theta_w,
      (uint64_t)(uintptr_t)P.k_eff, (uint64_t)(uintptr_t)P.e_node,
      (uint64_t)(uintptr_t)node_weight, (uint64_t)(uintptr_t)omega, bits(P.mu), bits(P.kT),
      (uint64_t)P.integrand, (uint64_t)p->block, (uint64_t)p->grid, (uint64_t)(uintptr_t)P.Wr,
      (uint64_t)(uintptr_t)P.Ur, (uint64_t)(uintptr_t)P.ret_slot};
  GraphCache& g = p->graphs[kind];
  if (!g.exec || g.key != key) {
    if (g.exec) {
      HIP_OR_FAIL(hipGraphExecDestroy(g.exec));
      g.exec = nullptr;
      g.key.clear();
    }
    HIP_OR_FAIL(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = forward_sequence(p, P, v_loc, node_weight, omega, s);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      g.exec = nullptr;
      return fail(SGQ_EHIP, std::string("graph capture of the forward launches: ") +
                                hipGetErrorString(e));
    }
    g.key = key;
  }
  HIP_OR_FAIL(hipGraphLaunch(g.exec, s));
  mark_retained(p, v_loc, P);
  return SGQ_OK;
}

extern "C" int rho_quadrature(sgq_plan* plan, const double* v_loc, const double* atom_R,
                              const double* proj_E, double mu, double kT, double* rho,
                              double* theta_w, int32_t* k_eff, void* stream) {
  int st = check_call(plan, v_loc, atom_R, proj_E, mu, kT);
  if (st != SGQ_OK) return st;
  if (!rho && plan->prob.n_nodes > 0) return fail(SGQ_EINVAL, "rho is null");
  LaunchParams P = base_params(plan, v_loc, atom_R, proj_E, mu, kT);
  P.rho = rho;
  P.theta_w = theta_w;
  P.k_eff = k_eff;
  P.integrand = 0;
  if (plan->schedule == SGQ_SCHEDULE_PLAIN) {
    if (theta_w) return fail(SGQ_EPLAN, "the plain schedule does not return the Gauss rule");
    hipStream_t s = (hipStream_t)stream;
    HIP_OR_FAIL(hipSetDevice(plan->device));
    P.slot_stride = (size_t)plan->kmax * plan->npad;
    HIP_OR_FAIL(launch_setup(P, plan->fp64, v_loc, plan->d_v, plan->d_chi, plan->d_g0, plan->d_vmax, s));
    plan->ret_valid = false;
    plan->tri_valid = false;
    HIP_OR_FAIL(launch_plain(P, plan->fp64, plan->h_center.data(), plan->h_hw.data(),
                             plan->h_depth.data(), plan->d_plain, s));
    plan->last = s;
    return SGQ_OK;
  }
  return run_forward(plan, 0, P, v_loc, nullptr, nullptr, (hipStream_t)stream);
}

extern "C" int sgq_plan_set_schedule(sgq_plan* plan, int schedule) {
  if (!plan) return fail(SGQ_EINVAL, "plan is null");
  if (schedule != SGQ_SCHEDULE_BATCHED && schedule != SGQ_SCHEDULE_PLAIN)
    return fail(SGQ_EINVAL, "unknown schedule");
  if (schedule == SGQ_SCHEDULE_PLAIN && !plan->d_plain) {
    // the plain schedule's scratch is allocated here, so that its compute calls allocate nothing
    HIP_OR_FAIL(hipSetDevice(plan->device));
    hipError_t e = dalloc(plan, &plan->d_plain, plain_scratch_bytes(plan->npad, plan->kmax, plan->fp64));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(SGQ_ENOMEM, std::string("plain schedule scratch: ") + hipGetErrorString(e));
    }
  }
  plan->schedule = schedule;
  return SGQ_OK;
}

extern "C" int sgq_fermi_level(sgq_plan* plan, const double* theta_w, const double* node_weight,
                               double n_electrons, double kT, double tol, double* result,
                               void* stream) {
  if (!plan) return fail(SGQ_EINVAL, "plan is null");
  if (plan->prob.n_nodes < 1) return fail(SGQ_EINVAL, "the plan has no nodes");
  if (!theta_w || !node_weight || !result) return fail(SGQ_EINVAL, "null argument");
  if (!(kT > 0.0) || !std::isfinite(kT)) return fail(SGQ_EINVAL, "kT must be finite and > 0");
  if (!(n_electrons > 0.0) || !std::isfinite(n_electrons))
    return fail(SGQ_EINVAL, "n_electrons must be finite and > 0");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(SGQ_EINVAL, "tol must be finite and > 0");
  if ((size_t)plan->prob.n_nodes * plan->kmax >= ((size_t)1 << 31))
    return fail(SGQ_EINVAL, "too many rule points for the Fermi-level kernel");
  hipStream_t s = (hipStream_t)stream;
  HIP_OR_FAIL(hipSetDevice(plan->device));
  HIP_OR_FAIL(launch_fermi_level(theta_w, node_weight, plan->prob.n_nodes, plan->kmax, n_electrons,
                                 kT, tol, result, plan->d_status, plan->d_fermi, s));
  plan->last = s;
  return SGQ_OK;
}

extern "C" int sgq_cluster_energy(sgq_plan* plan, const double* e_node,
                                  const int64_t* member_offset, const int32_t* member_node,
                                  int64_t n_members, int32_t n_esp, const double* esp_weight,
                                  double* fbar, double* energy, void* stream) {
  if (!plan) return fail(SGQ_EINVAL, "plan is null");
  if (plan->prob.n_nodes < 1) return fail(SGQ_EINVAL, "the plan has no nodes");
  if (n_esp < 1) return fail(SGQ_EINVAL, "n_esp must be >= 1");
  if (n_members < 1) return fail(SGQ_EINVAL, "n_members must be >= 1");
  if (!e_node || !member_offset || !member_node || !fbar) return fail(SGQ_EINVAL, "null argument");
  if (!energy != !esp_weight) return fail(SGQ_EINVAL, "energy and esp_weight go together");
  hipStream_t s = (hipStream_t)stream;
  HIP_OR_FAIL(hipSetDevice(plan->device));
  HIP_OR_FAIL(launch_cluster_energy(e_node, plan->prob.n_nodes, member_offset, member_node,
                                    n_members, n_esp, esp_weight, fbar, energy, plan->d_status,
                                    s));
  plan->last = s;
  return SGQ_OK;
}

// Frees the retained storage.
static void release_retained(sgq_plan* p) {
  for (void** a : {&p->d_Wr, &p->d_Ur}) {
    if (!*a) continue;
    (void)hipFree(*a);
    p->allocs.erase(std::remove(p->allocs.begin(), p->allocs.end(), *a), p->allocs.end());
    *a = nullptr;
  }
  p->retain = false;
  p->ret_nodes = 0;
}

extern "C" int sgq_plan_set_retain(sgq_plan* plan, int enable, int64_t max_bytes,
                                   int64_t* n_retained) {
  if (!plan) return fail(SGQ_EINVAL, "plan is null");
  if (n_retained) *n_retained = 0;
  if (max_bytes < 0) return fail(SGQ_EINVAL, "max_bytes < 0");
  plan->ret_valid = false;
  HIP_OR_FAIL(hipSetDevice(plan->device));
  HIP_OR_FAIL(hipDeviceSynchronize());   // no launch may still read the storage or its table
  release_retained(plan);
  if (!enable) return SGQ_OK;
  const int64_t nq = plan->prob.n_nodes;
  const size_t es = plan->fp64 ? 8 : 4;
  const size_t row_set = (size_t)plan->kmax * plan->npad * es;   // one node's basis (or U rows)
  int64_t m = nq;
  if (max_bytes > 0) m = std::min<int64_t>(nq, (int64_t)((size_t)max_bytes / (2 * row_set)));
  if (nq > 0 && m < 1)
    return fail(SGQ_EINVAL, "max_bytes holds no node's retained rows (" +
                                std::to_string(2 * row_set) + " bytes per node)");
  if (nq > 0) {
    if (!plan->d_ret_slot) {
      hipError_t e = dalloc(plan, &plan->d_ret_slot, sizeof(int32_t) * (size_t)nq);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SGQ_ENOMEM, std::string("retained-node table: ") + hipGetErrorString(e));
      }
    }
    // the first m nodes of the cost-sorted queue, the costliest to recompute
    std::vector<int32_t> slot((size_t)nq, -1);
    for (int64_t i = 0; i < m; ++i) slot[(size_t)plan->h_order[(size_t)i]] = (int32_t)i;
    HIP_OR_FAIL(hipMemcpy(plan->d_ret_slot, slot.data(), sizeof(int32_t) * (size_t)nq,
                          hipMemcpyHostToDevice));
    hipError_t e = dalloc(plan, &plan->d_Wr, (size_t)m * row_set);
    e = e ? e : dalloc(plan, &plan->d_Ur, (size_t)m * row_set);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      release_retained(plan);
      return fail(SGQ_ENOMEM, std::string("retained bases: ") + hipGetErrorString(e));
    }
  }
  plan->retain = true;
  plan->ret_nodes = m;
  if (n_retained) *n_retained = m;
  return SGQ_OK;
}

extern "C" int sgq_plan_set_graph(sgq_plan* plan, int enable) {
  if (!plan) return fail(SGQ_EINVAL, "plan is null");
  plan->use_graph = enable != 0;
  return SGQ_OK;
}

// ------------------------------------------------------------------ launch-shape autotuner
// Candidate launch shapes of the persistent forward kernel: workgroup size (lanes per
// node) and resident workgroups per CU.  Each is timed on a stratified sample of the
// plan's own nodes; the fastest is kept for the plan and cached per problem shape (in
// the process, and in the file named by SGQ_TUNE_CACHE when it is set).
namespace {
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune;
bool g_tune_file_read = false;

std::string tune_key(const sgq_plan* p) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) != hipSuccess) std::strcpy(prop.gcnArchName, "?");
  char buf[320];
  std::snprintf(buf, sizeof buf, "%s/cu%d/%s/npad%zu/kmax%d/proj%d/m%d", prop.gcnArchName, p->ncu,
                p->fp64 ? "f64" : "f32", p->npad, p->kmax, p->prob.n_proj, p->box_m);
  return buf;
}

void tune_file_read() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char* path = std::getenv("SGQ_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char key[320];
  int b, w;
  while (std::fscanf(f, "%319s %d %d", key, &b, &w) == 3) g_tune[key] = {b, w};
  std::fclose(f);
}

void tune_file_append(const std::string& key, int b, int w) {
  const char* path = std::getenv("SGQ_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d\n", key.c_str(), b, w);
  std::fclose(f);
}
}  // namespace

static int ensure_slots(sgq_plan* p, int slots) {
  if (slots <= p->slots) return SGQ_OK;
  const size_t es = p->fp64 ? 8 : 4;
  void *W = nullptr, *U = nullptr;
  hipError_t e = hipMalloc(&W, (size_t)slots * p->slot_stride * es);
  if (e == hipSuccess) e = hipMalloc(&U, (size_t)slots * p->npad * es);
  if (e != hipSuccess) {
    if (W) (void)hipFree(W);
    (void)hipGetLastError();
    return fail(SGQ_ENOMEM, "autotune: workspace for more resident workgroups");
  }
  HIP_OR_FAIL(hipDeviceSynchronize());
  for (GraphCache& g : p->graphs) {   // captured launches name the old workspace
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    g.key.clear();
  }
  for (void*& a : p->allocs) {
    if (a == p->d_W) { (void)hipFree(a); a = W; }
    else if (a == p->d_U) { (void)hipFree(a); a = U; }
  }
  p->d_W = W;
  p->d_U = U;
  p->slots = slots;
  return SGQ_OK;
}

extern "C" int sgq_plan_autotune(sgq_plan* plan, const double* v_loc, const double* atom_R,
                                 const double* proj_E, double mu, double kT, int sample_nodes,
                                 void* stream, int32_t* chosen) {
  int st = check_call(plan, v_loc, atom_R, proj_E, mu, kT);
  if (st != SGQ_OK) return st;
  if (sample_nodes < 1) return fail(SGQ_EINVAL, "sample_nodes must be >= 1");
  HIP_OR_FAIL(hipSetDevice(plan->device));
  plan->ret_valid = false;   // the timing launches overwrite sampled nodes' retained bases
  plan->tri_valid = false;   // and their stored tridiagonals
  hipStream_t s = (hipStream_t)stream;
  const int nq = plan->prob.n_nodes;
  std::vector<std::pair<int, int>> cand;
  if (plan->fp64) cand = {{256, 2}, {256, 1}};
  else cand = {{256, 2}, {256, 1}, {128, 3}, {128, 2}, {512, 1}};
  const std::string key = tune_key(plan);
  std::pair<int, int> best{plan->block, plan->grid / std::max(1, plan->ncu)};
  bool cached = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_file_read();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      best = it->second;
      cached = true;
    }
  }
  if (!cached && nq > 0) {
    int maxwpc = 0;
    for (auto& c : cand) maxwpc = std::max(maxwpc, c.second);
    st = ensure_slots(plan, std::min(nq, plan->ncu * maxwpc));
    if (st != SGQ_OK) return st;
    const int S = std::min(sample_nodes, nq);
    std::vector<int32_t> ids(S);
    for (int i = 0; i < S; ++i) ids[i] = plan->h_order[(size_t)i * nq / S];   // cost order kept
    int32_t* d_ids = nullptr;
    double* d_rho = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&d_ids, S * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&d_rho, (size_t)nq * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(d_ids, ids.data(), S * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    LaunchParams P = base_params(plan, v_loc, atom_R, proj_E, mu, kT);
    P.order = d_ids;
    P.n_nodes = S;
    P.rho = d_rho;
    // The candidates are timed in turn, round after round (the first round warms up), so
    // that a drift of the clocks while tuning favours none of them; each keeps its best
    // round.  A shape other than the first (256 lanes, two workgroups per CU: the plan's
    // default) is taken only when it beats that one by more than 1 %, about the spread of
    // these sample timings between shapes that are equally fast on the whole node set.
    std::vector<float> ms(cand.size(), 1e30f);
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
      for (size_t c = 0; c < cand.size() && e == hipSuccess; ++c) {
        const int grid = std::max(1, std::min(S, plan->ncu * cand[c].second));
        e = launch_setup(P, plan->fp64, v_loc, plan->d_v, plan->d_chi, plan->d_g0, plan->d_vmax, s);
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = launch_forward(P, plan->fp64, grid, cand[c].first, plan->kg, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (rep > 0) ms[c] = std::min(ms[c], t);
      }
    }
    size_t bi = 0;
    for (size_t c = 1; c < cand.size(); ++c)
      if (ms[c] < 0.99f * ms[0] && ms[c] < ms[bi]) bi = c;
    best = cand[bi];
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (d_ids) (void)hipFree(d_ids);
    if (d_rho) (void)hipFree(d_rho);
    if (e != hipSuccess) return fail(SGQ_EHIP, std::string("autotune: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    tune_file_append(key, best.first, best.second);
  }
  if (nq > 0) {
    st = ensure_slots(plan, std::min(nq, plan->ncu * best.second));
    if (st != SGQ_OK) return st;
  }
  plan->block = best.first;
  plan->grid = std::max(1, std::min(nq, plan->ncu * best.second));
  plan->tuned = true;
  if (chosen) {
    chosen[0] = best.first;
    chosen[1] = best.second;
  }
  return SGQ_OK;
}

extern "C" int band_energy(sgq_plan* plan, const double* v_loc, const double* atom_R,
                           const double* proj_E, const double* node_weight, double mu, double kT,
                           int integrand, double* e_node, double* omega, void* stream) {
  int st = check_call(plan, v_loc, atom_R, proj_E, mu, kT);
  if (st != SGQ_OK) return st;
  if (!omega || (plan->prob.n_nodes > 0 && (!node_weight || !e_node)))
    return fail(SGQ_EINVAL, "node_weight, e_node and omega are required");
  if (integrand < SGQ_BAND || integrand > SGQ_GRAND) return fail(SGQ_EINVAL, "bad integrand");
  LaunchParams P = base_params(plan, v_loc, atom_R, proj_E, mu, kT);
  P.e_node = e_node;
  P.integrand = integrand;
  return run_forward(plan, 1, P, v_loc, node_weight, omega, (hipStream_t)stream);
}

// Backward workspace, node cube offsets and the dV gather lists (sgq_plan_prepare_backward).
static int ensure_backward(sgq_plan* p) {
  if (p->bwd_ready) return SGQ_OK;
  if (p->kmax > backward_max_depth())
    return fail(SGQ_EPLAN, "backward supports Lanczos depths up to " +
                               std::to_string(backward_max_depth()));
  const int nq = p->prob.n_nodes;
  const size_t es = p->fp64 ? 8 : 4;
  // node cubes of the per-node dV contributions, each rounded up to 4 values so that every
  // cube starts 16-byte aligned (the reverse recurrence updates it with vector accesses)
  const std::vector<int64_t> off = cube_offsets(p->h_hw, (int64_t)p->n_grid);
  // gather lists: for every cell of the grid, the nodes (ascending) whose cube meets it
  std::vector<int32_t> cstart, clist;
  gather_lists(p->prob.n, p->h_center, p->h_hw, gather_cell(), cstart, clist);
  const int ncells = (int)cstart.size() - 1;
  {
    hipError_t e = hipSuccess;
    e = e ? e : dalloc(p, &p->d_cell_start, cstart.size() * 4);
    e = e ? e : dalloc(p, &p->d_cell_nodes, std::max<size_t>(1, clist.size()) * 4);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(SGQ_ENOMEM, "gather lists: " + std::string(hipGetErrorString(e)));
    }
    HIP_OR_FAIL(hipMemcpy(p->d_cell_start, cstart.data(), cstart.size() * 4, hipMemcpyHostToDevice));
    if (!clist.empty())
      HIP_OR_FAIL(hipMemcpy(p->d_cell_nodes, clist.data(), clist.size() * 4, hipMemcpyHostToDevice));
  }
  p->ncells = ncells;
  // two workgroups per CU (node state and adjoint scalars fit twice in a CU's LDS; the
  // eigenvector matrix of T lives in a global buffer per slot)
  p->grid_bwd = std::max(1, std::min(nq, 2 * p->ncu));
  // slot: the point-blocked basis (kmax rows), u_j then ubar_j (kmax rows), 3 adjoint rows
  p->bwd_slot_stride = (size_t)(2 * p->kmax + 3) * p->npad;
  hipError_t e = hipSuccess;
  e = e ? e : dalloc(p, &p->d_Wb, (size_t)p->grid_bwd * p->bwd_slot_stride * es);
  e = e ? e : dalloc(p, &p->d_Zb, (size_t)p->grid_bwd * backward_slot_doubles() * 8);
  e = e ? e : dalloc(p, &p->d_P, (size_t)std::max<int64_t>(1, off[nq]) * es);
  e = e ? e : dalloc(p, &p->d_cube_off, (size_t)(nq + 1) * 8);
  e = e ? e : dalloc(p, &p->d_dRp, (size_t)nq * kMaxNodeAtoms * 3 * 8);
  e = e ? e : dalloc(p, &p->d_dEp, (size_t)nq * kMaxNodeAtoms * 4 * 8);
  e = e ? e : dalloc(p, &p->d_node_atoms, (size_t)nq * (kMaxNodeAtoms + 1) * 4);
  // the eigensolve pre-pass: 16 one-wave workgroups per CU, each with the eigenvectors and
  // weighted divided differences of one node (2 kmax^2 doubles), and the per-node results
  p->grid_pre = std::max(1, std::min(nq, 16 * p->ncu));
  p->zpre_stride = 2 * (size_t)p->kmax * p->kmax;
  e = e ? e : dalloc(p, &p->d_zpre, (size_t)p->grid_pre * p->zpre_stride * 8);
  e = e ? e : dalloc(p, &p->d_tbar, (size_t)nq * 2 * p->kmax * 8);
  e = e ? e : dalloc(p, &p->d_tbar_k, (size_t)nq * 4);
  e = e ? e : dalloc(p, &p->d_border, (size_t)nq * 4);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SGQ_ENOMEM, std::string("backward workspace: ") + hipGetErrorString(e));
  }
  HIP_OR_FAIL(hipMemcpy(p->d_cube_off, off.data(), (nq + 1) * 8, hipMemcpyHostToDevice));
  // the backward's queue: the nodes of the 512-lane launch, then the rest, in cost order
  std::vector<int32_t> border(p->h_order);
  const auto mid = std::stable_partition(border.begin(), border.end(), [p](int32_t q) {
    return !p->fp64 && backward_wide_node(p->h_hw[(size_t)q]);
  });
  p->n_bwide = (int)(mid - border.begin());
  if (nq > 0)
    HIP_OR_FAIL(hipMemcpy(p->d_border, border.data(), (size_t)nq * 4, hipMemcpyHostToDevice));
  p->bwd_ready = true;
  return SGQ_OK;
}

extern "C" int band_energy_backward(sgq_plan* plan, const double* v_loc, const double* atom_R,
                                    const double* proj_E, const double* node_weight, double mu,
                                    double kT, int integrand, const double* grad_omega,
                                    double* dV, double* dR_nl, double* dE, void* stream) {
  int st = check_call(plan, v_loc, atom_R, proj_E, mu, kT);
  if (st != SGQ_OK) return st;
  if (!grad_omega || !dV || (plan->prob.n_nodes > 0 && !node_weight))
    return fail(SGQ_EINVAL, "grad_omega, dV and node_weight are required");
  if (integrand < SGQ_BAND || integrand > SGQ_GRAND) return fail(SGQ_EINVAL, "bad integrand");
  if (!plan->bwd_ready)
    return fail(SGQ_EPLAN, "the backward workspace is not prepared: call sgq_plan_prepare_backward");
  HIP_OR_FAIL(hipSetDevice(plan->device));
  hipStream_t s = (hipStream_t)stream;
  LaunchParams P = base_params(plan, v_loc, atom_R, proj_E, mu, kT);
  P.W = plan->d_Wb;
  P.zbuf = plan->d_Zb;
  P.slot_stride = plan->bwd_slot_stride;
  P.integrand = integrand;
  P.node_weight = node_weight;
  P.grad_omega = grad_omega;
  P.P_cube = plan->d_P;
  P.cube_offset = plan->d_cube_off;
  P.node_atoms = plan->d_node_atoms;
  P.dE_part = plan->d_dEp;
  P.dR_part = plan->d_dRp;
  // the bases retained by the last forward call, when it had these inputs (the backward
  // overwrites their u_j rows, so they serve one backward call)
  P.use_retained = plan->retain && plan->ret_valid && plan->ret_key[0] == v_loc &&
                   plan->ret_key[1] == atom_R && plan->ret_key[2] == proj_E;
  // this call's setup hashes the inputs' contents into the second entry; the kernel takes
  // the retained rows only when the forward call's hash agrees
  P.hash_slot = 1;
  plan->ret_valid = false;
  // the eigensolves of the nodes' tridiagonals run as a pass of their own when the last
  // forward launch stored them for these inputs (the pass checks the contents hash)
  const bool pre = plan->tri_valid && plan->tri_key[0] == v_loc && plan->tri_key[1] == atom_R &&
                   plan->tri_key[2] == proj_E;
  P.tbar = pre ? plan->d_tbar : nullptr;
  P.tbar_k = pre ? plan->d_tbar_k : nullptr;
  HIP_OR_FAIL(launch_setup(P, plan->fp64, v_loc, plan->d_v, plan->d_chi, plan->d_g0, plan->d_vmax, s));
  if (plan->prob.n_nodes > 0) {
    if (pre)
      HIP_OR_FAIL(launch_tbar(P, plan->grid_pre, plan->d_zpre, plan->zpre_stride, plan->d_tbar,
                              plan->d_tbar_k, s));
    // the nodes only the wide-plane march takes, with 512 lanes (one workgroup per CU);
    // then the others with 256 (two), from a fresh queue
    const int nq = plan->prob.n_nodes, nw = plan->n_bwide;
    if (nw > 0) {
      LaunchParams Pw = P;
      Pw.order = plan->d_border;
      Pw.n_nodes = nw;
      HIP_OR_FAIL(launch_backward(Pw, false, std::max(1, std::min(nw, plan->ncu)), 512, plan->kg, s));
    }
    if (nq > nw) {
      if (nw > 0) HIP_OR_FAIL(launch_queue_reset(P.queue, s));
      LaunchParams Pn = P;
      Pn.order = plan->d_border + nw;
      Pn.n_nodes = nq - nw;
      HIP_OR_FAIL(launch_backward(Pn, plan->fp64, std::max(1, std::min(nq - nw, plan->grid_bwd)),
                                  256, plan->kg, s));
    }
  }
  const bool have_proj = plan->prob.n_proj > 0 && plan->prob.n_atoms > 0;
  if (!have_proj) {
    HIP_OR_FAIL(launch_zero(dR_nl, dR_nl ? (size_t)plan->prob.n_atoms * 3 : 0, s));
    HIP_OR_FAIL(launch_zero(dE, dE ? (size_t)plan->prob.n_atoms * 4 : 0, s));
  }
  HIP_OR_FAIL(launch_backward_gather(P, plan->fp64, plan->d_cell_start, plan->d_cell_nodes,
                                     plan->ncells, dV, dR_nl, dE, s));
  plan->last = s;
  return SGQ_OK;
}

extern "C" int sgq_plan_prepare_backward(sgq_plan* plan) {
  if (!plan) return fail(SGQ_EINVAL, "plan is null");
  HIP_OR_FAIL(hipSetDevice(plan->device));
  return ensure_backward(plan);
}

extern "C" int sgq_vloc_gaussian_backward(sgq_plan* plan, const double* dV, const double* atom_R,
                                          double depth, double sigma, double cutoff_sigmas,
                                          double* dR, void* stream) {
  if (!plan || !dV || (plan->prob.n_atoms > 0 && (!atom_R || !dR)))
    return fail(SGQ_EINVAL, "null argument");
  if (!(sigma > 0.0) || !(cutoff_sigmas > 0.0) || !std::isfinite(depth))
    return fail(SGQ_EINVAL, "sigma and cutoff must be > 0, depth finite");
  HIP_OR_FAIL(hipSetDevice(plan->device));
  hipStream_t s = (hipStream_t)stream;
  HIP_OR_FAIL(launch_vloc_backward(dV, atom_R, plan->prob.n_atoms, plan->prob.n[0], plan->prob.n[1],
                                   plan->prob.n[2], plan->prob.h, depth, sigma, cutoff_sigmas, dR, s));
  plan->last = s;
  return SGQ_OK;
}

extern "C" int sgq_plan_status(sgq_plan* plan, int32_t* host_status) {
  if (!plan || !host_status) return fail(SGQ_EINVAL, "null argument");
  HIP_OR_FAIL(hipSetDevice(plan->device));
  if (plan->last) HIP_OR_FAIL(hipStreamSynchronize(plan->last));
  else HIP_OR_FAIL(hipDeviceSynchronize());
  int bits = 0;
  HIP_OR_FAIL(hipMemcpy(&bits, plan->d_status, 4, hipMemcpyDeviceToHost));
  *host_status = (bits & kStatusNonFinite) ? SGQ_ENONFINITE
                 : (bits & kStatusLimit)   ? SGQ_ELIMIT
                 : (bits & kStatusRange)   ? SGQ_ERANGE
                 : (bits & kStatusIndex)   ? SGQ_EINDEX
                                           : SGQ_OK;
  return SGQ_OK;
}
