// Predictor + corrector reconstruction of fields on the fine grid (Eq. eq:pc) with the
// correctors interpolated from the electronic sampling points (ESPs) by the linear
// shape functions of a tetrahedral mesh over them (Eq. phi_approx_scheme).
//
// Mesh object (sgq_fe_mesh_create): the ESPs sit on grid points, so every vertex has
// integer coordinates and so does every fine point; the signed volumes that decide
// whether a point lies in a tetrahedron are integers below 2^51 (axis extents are capped
// at 2^16) and are computed exactly in FP64.  The host orients every tetrahedron to
// positive volume, drops the zero-volume ones and files each kept tetrahedron under the
// cubic buckets its bounding box touches, in ascending tetrahedron order.  A location
// kernel then finds, once per mesh, the lowest-numbered tetrahedron holding each fine
// point (-1 if none).
//
// Reconstruction (sgq_fe_reconstruct), per call: one small kernel forms the correctors at
// the ESPs, fc_q = f_q - f0(r_q); the streaming kernel writes, for every fine point p,
// f_p = f0_p + sum_i lambda_i fc_{v_i} over the vertices of its tetrahedron, with the
// barycentric coordinates lambda_i = D_i / D recomputed from the exact volumes.  Points
// outside the mesh keep the predictor.  HBM traffic per fine point: the location (4 B)
// plus, per field, the predictor read and the result write (16 B).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "sgq.h"
#include "sgq_common.h"

namespace sgq {
int report_error(int code, const std::string& msg);
}

using sgq::report_error;

struct sgq_fe_mesh {
  int device = 0;
  int32_t n[3] = {0, 0, 0};
  int64_t npts = 0;
  int32_t n_esp = 0, n_tets = 0, n_kept = 0, max_fields = 0;
  int32_t bucket = 4, nb[3] = {1, 1, 1};
  int4* d_esp = nullptr;       // (x, y, z, linear index) per ESP
  uint2* d_xyz = nullptr;      // (x | y << 16, z) per ESP
  int32_t* d_lin = nullptr;    // linear fine-grid index per ESP
  int4* d_tet = nullptr;       // positively oriented vertex ids, caller's numbering
  int32_t* d_bstart = nullptr; // bucket CSR offsets
  int32_t* d_blist = nullptr;  // tetrahedron ids per bucket, ascending
  int32_t* d_loc = nullptr;    // tetrahedron of each fine point or -1
  double* d_corr = nullptr;    // correctors [n_esp][n_fields], fields interleaved
};

namespace sgq {
namespace {

constexpr int kFeBlock = 256;
constexpr uint32_t kXcds = 8;   // workgroups are dealt to the 8 XCDs round-robin by id

// Points [begin, end) of the slab of the grid that this workgroup's XCD owns, and the
// workgroup's first point and stride inside it.  Each XCD sweeps a contiguous slab, so its
// L2 only holds the mesh records of that slab.  The grid is a multiple of kXcds.
struct Slab {
  uint32_t p0, end, stride;
};

__device__ __forceinline__ Slab xcd_slab(uint32_t npts) {
  const uint32_t xcd = blockIdx.x % kXcds, lb = blockIdx.x / kXcds, nlb = gridDim.x / kXcds;
  const uint32_t chunk = (npts + kXcds - 1) / kXcds;
  const uint32_t begin = min(npts, xcd * chunk);
  Slab s;
  s.end = min(npts, begin + chunk);
  s.p0 = begin + lb * blockDim.x + threadIdx.x;
  s.stride = nlb * blockDim.x;
  return s;
}

// det[b - a, c - a, d - a] of integer points, exact in FP64 for coordinates below 2^16.
__device__ __forceinline__ double orient(double ax, double ay, double az, double bx, double by,
                                         double bz, double cx, double cy, double cz, double dx,
                                         double dy, double dz) {
  const double ux = bx - ax, uy = by - ay, uz = bz - az;
  const double vx = cx - ax, vy = cy - ay, vz = cz - az;
  const double wx = dx - ax, wy = dy - ay, wz = dz - az;
  return ux * (vy * wz - vz * wy) - uy * (vx * wz - vz * wx) + uz * (vx * wy - vy * wx);
}

// The four barycentric numerators of point (x, y, z) in tetrahedron t (each >= 0 inside a
// positively oriented tetrahedron; they sum to its volume det).
struct Bary {
  double d[4];
};

__device__ __forceinline__ Bary bary(const int4* __restrict__ esp, int4 t, double x, double y,
                                     double z) {
  const int4 a = esp[t.x], b = esp[t.y], c = esp[t.z], e = esp[t.w];
  const double ax = a.x, ay = a.y, az = a.z, bx = b.x, by = b.y, bz = b.z;
  const double cx = c.x, cy = c.y, cz = c.z, ex = e.x, ey = e.y, ez = e.z;
  Bary r;
  r.d[0] = orient(x, y, z, bx, by, bz, cx, cy, cz, ex, ey, ez);
  r.d[1] = orient(ax, ay, az, x, y, z, cx, cy, cz, ex, ey, ez);
  r.d[2] = orient(ax, ay, az, bx, by, bz, x, y, z, ex, ey, ez);
  r.d[3] = orient(ax, ay, az, bx, by, bz, cx, cy, cz, x, y, z);
  return r;
}

__global__ __launch_bounds__(kFeBlock) void fe_locate_kernel(
    const int4* __restrict__ esp, const int4* __restrict__ tet, const int32_t* __restrict__ bstart,
    const int32_t* __restrict__ blist, int nx, int ny, int nz, int bucket, int nbx, int nby,
    int32_t* __restrict__ loc) {
  const uint32_t ux = (uint32_t)nx, uy = (uint32_t)ny;
  const Slab sl = xcd_slab(ux * uy * (uint32_t)nz);
  for (uint32_t p = sl.p0; p < sl.end; p += sl.stride) {
    const uint32_t row = p / ux;
    const int ix = (int)(p - row * ux), iy = (int)(row % uy), iz = (int)(row / uy);
    const int b = ix / bucket + nbx * (iy / bucket + nby * (iz / bucket));
    const double x = ix, y = iy, z = iz;
    int32_t found = -1;
    for (int32_t i = bstart[b], e = bstart[b + 1]; i < e; ++i) {
      const int32_t t = blist[i];
      const Bary r = bary(esp, tet[t], x, y, z);
      if (r.d[0] >= 0.0 && r.d[1] >= 0.0 && r.d[2] >= 0.0 && r.d[3] >= 0.0) {
        found = t;
        break;
      }
    }
    loc[p] = found;
  }
}

// fc_q = f_q - f0(r_q) for every field, one ESP per lane: the ESP's fine-grid index is read
// once for all F fields (from its own packed array), and its correctors are stored ESP-major
// in one contiguous write (the fields of one ESP are adjacent, so the reconstruction fetches
// them with one load).  f_q comes field-major, [F][n_esp].
template <int F>
__global__ __launch_bounds__(kFeBlock) void fe_corrector_kernel(
    const int32_t* __restrict__ lin, int n_esp, int64_t npts,
    const double* __restrict__ esp_values, const double* __restrict__ predictor,
    double* __restrict__ corr) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n_esp; q += gridDim.x * blockDim.x) {
    const int64_t p = lin[q];
    double c[F];
#pragma unroll
    for (int f = 0; f < F; ++f) c[f] = esp_values[(int64_t)f * n_esp + q] - predictor[f * npts + p];
    double* b = corr + (int64_t)q * F;
    if constexpr (F == 2 || F == 4) {
#pragma unroll
      for (int h = 0; h < F / 2; ++h) reinterpret_cast<double2*>(b)[h] = make_double2(c[2 * h], c[2 * h + 1]);
    } else {
#pragma unroll
      for (int f = 0; f < F; ++f) b[f] = c[f];
    }
  }
}

template <int F>
__device__ __forceinline__ void load_corr(const double* __restrict__ corr, int q, double* c) {
  const double* b = corr + (int64_t)q * F;
  if constexpr (F == 2 || F == 4) {
#pragma unroll
    for (int h = 0; h < F / 2; ++h) {
      const double2 v = reinterpret_cast<const double2*>(b)[h];
      c[2 * h] = v.x;
      c[2 * h + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int f = 0; f < F; ++f) c[f] = b[f];
  }
}

// One fine point per lane.  D_i are the exact barycentric numerators; 1/D is the hardware
// reciprocal refined by two Newton steps (error below an ulp of the quotient).
template <int F>
__global__ __launch_bounds__(kFeBlock) void fe_reconstruct_kernel(
    const uint2* __restrict__ xyz, const int4* __restrict__ tet, const int32_t* __restrict__ loc,
    int nx, int ny, int64_t npts, const double* __restrict__ corr,
    const double* __restrict__ predictor, double* __restrict__ out) {
  const uint32_t ux = (uint32_t)nx, uy = (uint32_t)ny;
  const Slab sl = xcd_slab((uint32_t)npts);
  for (uint32_t p = sl.p0; p < sl.end; p += sl.stride) {
    const int32_t t = loc[p];
    double f0[F];
#pragma unroll
    for (int f = 0; f < F; ++f) f0[f] = __builtin_nontemporal_load(predictor + f * npts + p);
    if (t >= 0) {
      const uint32_t row = p / ux;
      const double x = (double)(p - row * ux), y = (double)(row % uy), z = (double)(row / uy);
      const int4 v = tet[t];
      const int vid[4] = {v.x, v.y, v.z, v.w};
      double vx[4], vy[4], vz[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint2 e = xyz[vid[i]];
        vx[i] = (double)(e.x & 0xffffu);
        vy[i] = (double)(e.x >> 16);
        vz[i] = (double)e.y;
      }
      // edges e_k = v_k - v_0 and r = x - v_0; with n_1 = e_2 x e_3, n_2 = e_3 x e_1,
      // n_3 = e_1 x e_2 the numerators are D_k = r . n_k (k = 1..3), D = e_1 . n_1 and
      // D_0 = D - D_1 - D_2 - D_3: integers below 2^51, exact in FP64
      const double e1x = vx[1] - vx[0], e1y = vy[1] - vy[0], e1z = vz[1] - vz[0];
      const double e2x = vx[2] - vx[0], e2y = vy[2] - vy[0], e2z = vz[2] - vz[0];
      const double e3x = vx[3] - vx[0], e3y = vy[3] - vy[0], e3z = vz[3] - vz[0];
      const double rx = x - vx[0], ry = y - vy[0], rz = z - vz[0];
      const double n1x = e2y * e3z - e2z * e3y, n1y = e2z * e3x - e2x * e3z, n1z = e2x * e3y - e2y * e3x;
      const double n2x = e3y * e1z - e3z * e1y, n2y = e3z * e1x - e3x * e1z, n2z = e3x * e1y - e3y * e1x;
      const double n3x = e1y * e2z - e1z * e2y, n3y = e1z * e2x - e1x * e2z, n3z = e1x * e2y - e1y * e2x;
      const double D = e1x * n1x + e1y * n1y + e1z * n1z;
      double d[4];
      d[1] = rx * n1x + ry * n1y + rz * n1z;
      d[2] = rx * n2x + ry * n2y + rz * n2z;
      d[3] = rx * n3x + ry * n3y + rz * n3z;
      d[0] = D - d[1] - d[2] - d[3];
      double r = __builtin_amdgcn_rcp(D);
      r = fma(r, fma(-D, r, 1.0), r);
      r = fma(r, fma(-D, r, 1.0), r);
      double acc[F];
#pragma unroll
      for (int f = 0; f < F; ++f) acc[f] = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double c[F];
        load_corr<F>(corr, vid[i], c);
#pragma unroll
        for (int f = 0; f < F; ++f) acc[f] = fma(d[i], c[f], acc[f]);
      }
#pragma unroll
      for (int f = 0; f < F; ++f) f0[f] = fma(acc[f], r, f0[f]);
    }
#pragma unroll
    for (int f = 0; f < F; ++f) __builtin_nontemporal_store(f0[f], out + f * npts + p);
  }
}

int fe_grid_full(int64_t work) {
  const int64_t blocks = std::max<int64_t>(1, (work + kFeBlock - 1) / kFeBlock);
  return (int)((blocks + kXcds - 1) / kXcds * kXcds);
}

int fe_grid(int64_t work) {
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int64_t blocks = (work + kFeBlock - 1) / kFeBlock;
  const int64_t g = std::max<int64_t>(1, std::min<int64_t>(blocks, (int64_t)ncu * 16));
  return (int)((g + kXcds - 1) / kXcds * kXcds);
}

void free_mesh(sgq_fe_mesh* m) {
  (void)hipFree(m->d_esp);
  (void)hipFree(m->d_xyz);
  (void)hipFree(m->d_lin);
  (void)hipFree(m->d_tet);
  (void)hipFree(m->d_bstart);
  (void)hipFree(m->d_blist);
  (void)hipFree(m->d_loc);
  (void)hipFree(m->d_corr);
  delete m;
}

}  // namespace
}  // namespace sgq

#define FE_HIP(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) {                                                                \
      sgq::free_mesh(m);                                                                   \
      return report_error(SGQ_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    }                                                                                      \
  } while (0)

extern "C" int sgq_fe_mesh_create(const int32_t n[3], const int64_t* esp_center, int32_t n_esp,
                                  const int32_t* tets, int32_t n_tets, int32_t max_fields,
                                  sgq_fe_mesh** out) {
  if (!out) return report_error(SGQ_EINVAL, "out is null");
  *out = nullptr;
  // host geometry: ESP coordinates, oriented tetrahedra, bucket lists (host.cpp)
  sgq::FeGeometry geo;
  int st = sgq::fe_geometry(n, esp_center, n_esp, tets, n_tets, max_fields, &geo);
  if (st != SGQ_OK) return st;
  const int64_t npts = (int64_t)n[0] * n[1] * n[2];
  const int32_t kept = geo.kept;
  const int bucket = geo.bucket;
  const int* nb = geo.nb;
  // the [n][4] int32 arrays have the layout of int4 records
  static_assert(sizeof(int4) == 4 * sizeof(int32_t), "int4 records");
  const std::vector<int32_t>& bstart = geo.bstart;
  const std::vector<int32_t>& blist = geo.blist;
  const size_t ntet = geo.tet.size() / 4;
  sgq_fe_mesh* m = new sgq_fe_mesh;
  for (int a = 0; a < 3; ++a) {
    m->n[a] = n[a];
    m->nb[a] = nb[a];
  }
  m->npts = npts;
  m->n_esp = n_esp;
  m->n_tets = n_tets;
  m->n_kept = kept;
  m->max_fields = max_fields;
  m->bucket = bucket;
  FE_HIP(hipGetDevice(&m->device));
  FE_HIP(hipMalloc(&m->d_esp, sizeof(int4) * n_esp));
  FE_HIP(hipMalloc(&m->d_xyz, sizeof(uint2) * n_esp));
  FE_HIP(hipMalloc(&m->d_lin, sizeof(int32_t) * n_esp));
  FE_HIP(hipMalloc(&m->d_tet, sizeof(int4) * ntet));
  FE_HIP(hipMalloc(&m->d_bstart, sizeof(int32_t) * bstart.size()));
  FE_HIP(hipMalloc(&m->d_blist, sizeof(int32_t) * blist.size()));
  FE_HIP(hipMalloc(&m->d_loc, sizeof(int32_t) * npts));
  FE_HIP(hipMalloc(&m->d_corr, sizeof(double) * max_fields * (size_t)n_esp));
  FE_HIP(hipMemcpy(m->d_esp, geo.esp.data(), sizeof(int4) * n_esp, hipMemcpyHostToDevice));
  std::vector<uint2> packed(n_esp);
  std::vector<int32_t> lin(n_esp);
  for (int32_t q = 0; q < n_esp; ++q) {
    const int32_t* e = geo.esp.data() + 4 * (size_t)q;
    packed[q] = make_uint2((uint32_t)e[0] | ((uint32_t)e[1] << 16), (uint32_t)e[2]);
    lin[q] = e[3];
  }
  FE_HIP(hipMemcpy(m->d_xyz, packed.data(), sizeof(uint2) * n_esp, hipMemcpyHostToDevice));
  FE_HIP(hipMemcpy(m->d_lin, lin.data(), sizeof(int32_t) * n_esp, hipMemcpyHostToDevice));
  FE_HIP(hipMemcpy(m->d_tet, geo.tet.data(), sizeof(int4) * ntet, hipMemcpyHostToDevice));
  FE_HIP(hipMemcpy(m->d_bstart, bstart.data(), sizeof(int32_t) * bstart.size(), hipMemcpyHostToDevice));
  FE_HIP(hipMemcpy(m->d_blist, blist.data(), sizeof(int32_t) * blist.size(), hipMemcpyHostToDevice));
  hipLaunchKernelGGL(sgq::fe_locate_kernel, dim3(sgq::fe_grid(npts)), dim3(sgq::kFeBlock), 0, 0,
                     m->d_esp, m->d_tet, m->d_bstart, m->d_blist, n[0], n[1], n[2], bucket, nb[0],
                     nb[1], m->d_loc);
  FE_HIP(hipGetLastError());
  FE_HIP(hipDeviceSynchronize());
  *out = m;
  return SGQ_OK;
}

extern "C" int sgq_fe_mesh_destroy(sgq_fe_mesh* mesh) {
  if (!mesh) return SGQ_OK;
  (void)hipSetDevice(mesh->device);
  (void)hipDeviceSynchronize();
  sgq::free_mesh(mesh);
  return SGQ_OK;
}

extern "C" int sgq_fe_mesh_info(const sgq_fe_mesh* mesh, int64_t* info) {
  if (!mesh || !info) return report_error(SGQ_EINVAL, "null argument");
  info[0] = mesh->npts;
  info[1] = mesh->n_esp;
  info[2] = mesh->n_tets;
  info[3] = mesh->n_kept;
  info[4] = mesh->bucket;
  return SGQ_OK;
}

extern "C" int sgq_fe_mesh_location(sgq_fe_mesh* mesh, int32_t* loc, void* stream) {
  if (!mesh || !loc) return report_error(SGQ_EINVAL, "null argument");
  hipError_t e = hipSetDevice(mesh->device);
  if (e == hipSuccess)
    e = hipMemcpyAsync(loc, mesh->d_loc, sizeof(int32_t) * mesh->npts, hipMemcpyDeviceToDevice,
                       (hipStream_t)stream);
  if (e != hipSuccess) return report_error(SGQ_EHIP, hipGetErrorString(e));
  return SGQ_OK;
}

extern "C" int sgq_fe_reconstruct(sgq_fe_mesh* mesh, int32_t n_fields, const double* esp_values,
                                  const double* predictor, double* out, void* stream) {
  if (!mesh) return report_error(SGQ_EINVAL, "mesh is null");
  if (n_fields < 1 || n_fields > mesh->max_fields)
    return report_error(SGQ_EINVAL, "n_fields must be in [1, max_fields of the mesh]");
  if (!esp_values || !predictor || !out) return report_error(SGQ_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSetDevice(mesh->device);
  if (e != hipSuccess) return report_error(SGQ_EHIP, hipGetErrorString(e));
  const dim3 cgrid(sgq::fe_grid(mesh->n_esp)), grid(sgq::fe_grid_full(mesh->npts)),
      block(sgq::kFeBlock);
  switch (n_fields) {
#define FE_CASE(F)                                                                               \
  case F:                                                                                        \
    hipLaunchKernelGGL(sgq::fe_corrector_kernel<F>, cgrid, block, 0, s, mesh->d_lin,             \
                       mesh->n_esp, mesh->npts, esp_values, predictor, mesh->d_corr);            \
    hipLaunchKernelGGL(sgq::fe_reconstruct_kernel<F>, grid, block, 0, s, mesh->d_xyz, mesh->d_tet, \
                       mesh->d_loc, mesh->n[0], mesh->n[1], mesh->npts, mesh->d_corr, predictor,  \
                       out);                                                                      \
    break;
    FE_CASE(1)
    FE_CASE(2)
    FE_CASE(3)
    FE_CASE(4)
#undef FE_CASE
  }
  e = hipGetLastError();
  if (e != hipSuccess) return report_error(SGQ_EHIP, hipGetErrorString(e));
  return SGQ_OK;
}
