/*
 * sgq.h - C ABI of the MI355X spectral Gauss-quadrature density library (libsgq.so).
 *
 * What the library computes (paper: Sec. "Density Functional Theory"):
 *   For every node p of a uniform periodic finite-difference grid, the K-point Gauss
 *   rule (lambda_k, w_k) of the spectral measure of the Kohn-Sham Hamiltonian H
 *   contracted with the orthonormal FD basis function eta_p (Eq. eq:9), obtained by
 *   a K-step Lanczos iteration started from eta_p; from it the density
 *   rho_p = 2 h^-3 sum_k w_k g(lambda_k) (Eq. Eqn:LSSGQ:Electron_density:GQ) with the
 *   Fermi-Dirac occupation g of Eq. eq:dm, the per-node energy term
 *   e_p = 2 sum_k w_k F(lambda_k) (band and entropy terms of Eq. eq:tot) and the
 *   node-weighted sum Omega = sum_q n_q e_q (Eq. eq:free_cg), plus the adjoint of
 *   Omega with respect to the local potential, projector energies and atom positions.
 *
 *   H = -1/2 Lap_6 + V_loc + V_nl, Lap_6 the sixth-order central FD Laplacian (axis
 *   stencil), V_loc a grid potential, V_nl = sum_J sum_l |chi_Jl> E_Jl <chi_Jl| with
 *   <chi|v> = h^3 sum_x chi(x) v(x) and four Gaussian projectors per atom
 *   (s, px, py, pz) of width proj_rg and smooth cutoff proj_rc (bohr).
 *   Node truncation: H_q is H restricted to the cube of side 2R+1 around the node
 *   (grid indices wrap periodically, Dirichlet zero outside); R = -1 keeps the whole
 *   periodic grid.
 *
 * Conventions
 *   - Grid arrays are [z][y][x] with x fastest: linear index ix + nx*(iy + ny*iz).
 *   - Every array argument of a compute call is a DEVICE pointer owned by the caller,
 *     contiguous, of the stated type and length.  Host arrays are passed only to
 *     sgq_plan_create, sgq_fe_mesh_create and the host-only helpers (sgq_cluster_build,
 *     sgq_validate, sgq_gauss_rule_host).
 *   - Compute calls are asynchronous on `stream` (a hipStream_t; NULL = default
 *     stream).  Inputs must stay valid until the stream reaches the call.  They allocate
 *     no device memory and do not synchronise: everything they need is allocated by the
 *     synchronous set-up calls (sgq_plan_create, sgq_plan_prepare_backward,
 *     sgq_plan_set_schedule, sgq_plan_set_retain, sgq_plan_autotune, the mesh and solver
 *     constructors), which report SGQ_ENOMEM.  (The HIP runtime itself sets up a stream's
 *     kernel-argument buffers, and a kernel's private memory, on their first launches.)
 *   - Every function returns an sgq_status and never throws.  Argument errors found
 *     on the host are returned before anything is launched; errors found by the GPU
 *     (non-finite input, a node touching more atoms than the library supports) are
 *     latched in the plan and reported by sgq_plan_status.
 *   - A plan is not thread-safe: calls on one plan must be serialised by the caller
 *     (they share the plan's workspace).
 */
#ifndef SGQ_H
#define SGQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SGQ_OK = 0,
  SGQ_EINVAL = -1,      /* invalid argument (null pointer, bad size, kT <= 0, ...) */
  SGQ_ENOMEM = -2,      /* device allocation failed (set-up calls only) */
  SGQ_EHIP = -3,        /* a HIP runtime call failed */
  SGQ_EPLAN = -4,       /* the call does not match the plan (e.g. no projectors planned) */
  SGQ_ENONFINITE = -5,  /* device status: NaN/Inf in an input */
  SGQ_ELIMIT = -6,      /* device status: a node overlaps more atoms than supported */
  SGQ_ERANGE = -7,      /* device status: no Fermi level for the requested electron count */
  SGQ_EINDEX = -8       /* device status: a cluster list entry outside the plan's nodes */
} sgq_status;

enum { SGQ_FP64 = 0, SGQ_FP32 = 1 };           /* storage / matvec precision */
enum { SGQ_BAND = 0, SGQ_FREE = 1, SGQ_GRAND = 2 };
enum { SGQ_SCHEDULE_BATCHED = 0, SGQ_SCHEDULE_PLAIN = 1 };

/* Integrands F of e_p = 2 sum_k w_k F(lambda_k), x = (lambda - mu)/kT, g = 1/(1+e^x):
 *   SGQ_BAND  F = lambda g                                  (first term of Eq. eq:tot)
 *   SGQ_FREE  F = lambda g + kT [g ln g + (1-g) ln(1-g)]    (Mermin free energy)
 *   SGQ_GRAND F = -kT ln(1 + e^-x)                          (grand potential)      */

typedef struct {
  int32_t n[3];          /* global grid points (nx, ny, nz), each >= 1 */
  double h;              /* grid spacing, bohr, > 0 */
  int32_t n_atoms;       /* M >= 0 */
  int32_t n_proj;        /* 0 (local potential only) or 4 (s, px, py, pz) */
  double proj_rc;        /* projector cutoff radius, bohr (> 0 when n_proj = 4) */
  double proj_rg;        /* projector Gaussian width, bohr (> 0 when n_proj = 4) */
  int32_t n_nodes;       /* Nq >= 0 */
  int32_t precision;     /* SGQ_FP64 or SGQ_FP32 (dots, tridiagonal and quadrature are FP64) */
} sgq_problem;

typedef struct sgq_plan sgq_plan;

/* Create a plan for a fixed grid and node set.  Host arrays of length n_nodes:
 *   center[q]     linear grid index of node q, in [0, nx*ny*nz)
 *   half_width[q] R_q >= 0 (cube side 2R_q+1 <= min(n) - 6) or -1 (whole periodic grid)
 *   depth[q]      Lanczos depth K_q in [1, 128]
 * Sorts the nodes by cost for the persistent launch and allocates the device
 * workspace (SGQ_ENOMEM if that fails).  Synchronous.  *out receives the plan. */
int sgq_plan_create(const sgq_problem* prob, const int64_t* center, const int32_t* half_width,
                    const int32_t* depth, sgq_plan** out);

int sgq_plan_destroy(sgq_plan* plan);

/* Density at every node.
 *   v_loc   [nz*ny*nx] double   local potential, Ha
 *   atom_R  [M*3]      double   atom positions (x, y, z), bohr; NULL allowed when M = 0
 *   proj_E  [M*4]      double   projector energies, Ha; NULL allowed when n_proj = 0
 *   mu, kT                      Fermi level and temperature, Ha (kT > 0)
 *   rho     [Nq]       double   out: rho_q, electrons / bohr^3
 *   theta_w [Nq*Kmax*2] double  out (optional, NULL): (lambda_k, w_k) of node q at
 *                               [(q*Kmax + k)*2], zero beyond K_eff; Kmax = max depth
 *   k_eff   [Nq]       int32    out (optional, NULL): nodes of the rule (< K_q after a
 *                               Lanczos breakdown, when the rule is exact)           */
int rho_quadrature(sgq_plan* plan, const double* v_loc, const double* atom_R,
                   const double* proj_E, double mu, double kT, double* rho, double* theta_w,
                   int32_t* k_eff, void* stream);

/* Per-node energy term and the weighted sum (Eq. eq:tot first and entropy terms,
 * Eq. eq:free_cg).
 *   node_weight [Nq] double   n_q
 *   integrand            SGQ_BAND, SGQ_FREE or SGQ_GRAND
 *   e_node  [Nq] double       out: e_q = 2 sum_k w_k F(lambda_k), Ha
 *   omega   [1]  double       out: Omega = sum_q n_q e_q, summed in a fixed order     */
int band_energy(sgq_plan* plan, const double* v_loc, const double* atom_R,
                const double* proj_E, const double* node_weight, double mu, double kT,
                int integrand, double* e_node, double* omega, void* stream);

/* Backward workspace of a plan: the per-workgroup adjoint slots, the per-node dV cubes
 * (one cube of the node's points per node: 15.9 GB for 110592 nodes of 33^3 points in
 * FP32), the per-node atom partials, the lists that gather the cubes into dV, and the
 * eigensolve pre-pass's buffers (per node 2 K_max doubles of alphabar / betabar; per
 * pre-pass workgroup, 16 per CU, 2 K_max^2 doubles), and the backward's node
 * queue (FP32 cubes of 37 to 49 points first, reversed with 512 lanes per node, then the
 * others, with 256).  Allocates and uploads them (host
 * geometry, hipMalloc, blocking copies), so it is synchronous; call it once before the
 * first band_energy_backward.  Returns SGQ_ENOMEM when the workspace does not fit,
 * SGQ_EPLAN when the plan's depth exceeds the adjoint's (128, every depth a plan
 * accepts); calling it again is a no-op. */
int sgq_plan_prepare_backward(sgq_plan* plan);

/* Adjoint of Omega (reverse mode through the Lanczos recurrence; the Lanczos vectors
 * of each node are recomputed from the start vector, the only checkpoint kept, unless the
 * forward call retained them, see sgq_plan_set_retain).  When the plan's last forward call
 * (rho_quadrature or band_energy over all nodes) saw the same inputs, the eigensolves of
 * the nodes' tridiagonals run as a pre-pass over the tridiagonals it stored.  Requires
 * sgq_plan_prepare_backward (SGQ_EPLAN otherwise); the call itself allocates nothing and
 * does not synchronise: it only enqueues kernels on `stream`.
 *   grad_omega [1] double        upstream dL/dOmega
 *   dV    [nz*ny*nx] double      out: dL/dV_loc(x)
 *   dR_nl [M*3] double           out: dL/dR_J through the projectors (NULL allowed when
 *                                n_proj = 0); the local-potential part is
 *                                sgq_vloc_gaussian_backward of dV
 *   dE    [M*4] double           out (optional, NULL): dL/dE_Jl                       */
int band_energy_backward(sgq_plan* plan, const double* v_loc, const double* atom_R,
                         const double* proj_E, const double* node_weight, double mu,
                         double kT, int integrand, const double* grad_omega, double* dV,
                         double* dR_nl, double* dE, void* stream);

/* Chain rule through the Gaussian local potential
 *   V(x) = depth sum_J sum_images exp(-|x - R_J - L m|^2 / (2 sigma^2))
 * keeping image terms with distance <= cutoff_sigmas * sigma:
 *   dR[J] += sum_x dV(x) dV(x)/dR_J.
 *   dV [nz*ny*nx] double, atom_R [M*3] double, dR [M*3] double (accumulated into). */
int sgq_vloc_gaussian_backward(sgq_plan* plan, const double* dV, const double* atom_R,
                               double depth, double sigma, double cutoff_sigmas, double* dR,
                               void* stream);

/* Execution schedule of rho_quadrature on this plan.
 *   SGQ_SCHEDULE_BATCHED (default): all nodes in one persistent launch, one workgroup per
 *                        node, the reorthogonalised Lanczos step fused as described above.
 *   SGQ_SCHEDULE_PLAIN:  one node after another, every Lanczos step as grid-wide kernels
 *                        (classical Gram-Schmidt against all earlier vectors); the
 *                        per-node GPU baseline.  Same precision and depth; theta_w must be
 *                        NULL.  Its scratch is allocated by this call (synchronous;
 *                        SGQ_ENOMEM if it does not fit, and the schedule is unchanged), so
 *                        the compute calls allocate nothing.
 * Returns SGQ_EINVAL for an unknown schedule. */
int sgq_plan_set_schedule(sgq_plan* plan, int schedule);

/* Fermi level of stored Gauss rules (Eq. Eqn:LSSGQ:Fermi_level:GQ, with the node weights
 * of Eq. eq:free_cg): the mu at which the electron count
 *   N(mu) = 2 sum_q n_q sum_k w_k g(lambda_k; mu),  g = 1/(1 + exp((lambda - mu)/kT)),
 * equals n_electrons.  The rules are mu- and kT-independent, so this needs no new Lanczos
 * run: theta_w is the rule output of rho_quadrature on this plan.
 *   theta_w     [Nq*Kmax*2] double  device: (lambda_k, w_k) per node; entries with w_k = 0
 *                                   (beyond K_eff) are ignored
 *   node_weight [Nq]        double  device: n_q
 *   n_electrons, kT                 > 0; tol > 0: stop when |N(mu) - n_electrons| <=
 *                                   tol * n_electrons
 *   result      [3]         double  device out: mu, N(mu), number of Newton/bisection steps
 * Safeguarded Newton iteration (at most 64 steps) on a bracket spanning every rule point by
 * 60 kT; every step sums over the rule points on the whole device, in a fixed order (bitwise
 * reproducible), through the plan's own small workspace.  An electron count
 * outside (0, 2 sum_q n_q sum_k w_k) latches SGQ_ERANGE (result = NaN), a non-finite rule
 * SGQ_ENONFINITE; both are read with sgq_plan_status.  Asynchronous on `stream`. */
int sgq_fermi_level(sgq_plan* plan, const double* theta_w, const double* node_weight,
                    double n_electrons, double kT, double tol, double* result, void* stream);

/* The Fermi-level solve of sgq_fermi_level without a plan and without allocating: for
 * callers that cannot allocate device memory (code under HIP graph capture, tight
 * self-consistency loops, harnesses that forbid hipMalloc).  Its state and partial sums
 * (16 + 4 x 512 doubles) and status word live in a file-scope device array of the library,
 * one copy per GPU, held until the process ends; the first call on a GPU looks up that
 * array's address once.  The call enqueues the same kernels as sgq_fermi_level on `stream`
 * and nothing else (no allocation, no memset, no synchronisation).
 *   theta_w [n_nodes*kmax*2] double, node_weight [n_nodes] double: device inputs as for
 *                             sgq_fermi_level (kmax = the rule's stride per node)
 *   n_electrons, kT, tol      as for sgq_fermi_level
 *   result [3] double         device out: mu, N(mu), steps
 *   status [1] int32          device out: SGQ_OK, SGQ_ERANGE (no level for the count) or
 *                             SGQ_ENONFINITE (a non-finite rule or weight), written by the
 *                             last kernel of the call
 * Returns SGQ_EINVAL for a null pointer, n_nodes or kmax below 1, n_nodes * kmax of 2^31 or
 * more rule points, or a bad scalar; SGQ_EHIP when a launch fails.  Every call on one GPU
 * shares the array: calls that overlap on a GPU (other host threads, other streams) race
 * and must be serialised by the caller. */
int sgq_fermi_level_noalloc(const double* theta_w, const double* node_weight, int32_t n_nodes,
                            int32_t kmax, double n_electrons, double kT, double tol,
                            double* result, int32_t* status, void* stream);

/* Clusters of the energy sampling (Eq. eq:free_cg_sampling), host only.  C_q is the set
 * of grid points within distance `radius` (bohr) of energy sampling point (ESP) q on the
 * periodic grid (minimum-image distance; a point is inside when its squared distance in
 * grid units is <= (radius/h)^2 (1 + 1e-9), so a radius equal to a lattice distance keeps
 * that shell).  The clusters are merged into one ascending node list, so a point shared by
 * several clusters is evaluated once; build a plan on that list and feed its band_energy
 * e_node to sgq_cluster_energy.  All arrays are HOST arrays.
 *   n [3], h              grid extents and spacing, as in sgq_problem
 *   esp_center [n_esp]    int64  linear grid index of each ESP
 *   radius                >= 0
 *   esp_weight [n_esp]    double optional: n_q, needed only for node_weight
 *   node_capacity, member_capacity   lengths of the output arrays below
 *   node_center [Nn]      int64  out (optional): ascending linear indices of the merged nodes
 *   node_esp [Nn]         int32  out (optional): lowest ESP whose cluster holds the node
 *   node_weight [Nn]      double out (optional): sum over clusters q holding the node of
 *                         n_q / |C_q|, so that sum_p node_weight_p e_p = sum_q n_q Fbar_q
 *                         and band_energy / band_energy_backward with these weights give
 *                         the cluster-sampled energy and its gradient
 *   member_offset [n_esp+1] int64 out (optional): CSR offsets of the clusters
 *   member_node [Nm]      int32  out (optional): position in node_center of each member,
 *                         ascending within a cluster
 *   n_nodes, n_members    int64  out (required): Nn and Nm
 * Call once with the optional outputs NULL to get the counts.  A capacity below the
 * count returns SGQ_EINVAL (the counts are still written).  Every cluster holds its ESP,
 * so no cluster is empty. */
int sgq_cluster_build(const int32_t n[3], double h, const int64_t* esp_center, int32_t n_esp,
                      double radius, const double* esp_weight, int64_t node_capacity,
                      int64_t member_capacity, int64_t* node_center, int32_t* node_esp,
                      double* node_weight, int64_t* member_offset, int32_t* member_node,
                      int64_t* n_nodes, int64_t* n_members);

/* Cluster-sampled energy (Eq. eq:free_cg with the cluster averages of Eq.
 * eq:free_cg_sampling): Fbar_q = (1/|C_q|) sum_{p in C_q} e_p and
 * energy = sum_q n_q Fbar_q.  Device arrays:
 *   e_node [Nq]            double  per-node energies of this plan (band_energy output)
 *   member_offset [n_esp+1] int64, member_node [n_members] int32: clusters as written
 *                          by sgq_cluster_build (positions in the plan's node list)
 *   esp_weight [n_esp]     double  n_q (optional, NULL only together with energy)
 *   fbar [n_esp]           double  out
 *   energy [1]             double  out (optional)
 * One wavefront per cluster and a one-workgroup weighted sum, both in a fixed order
 * (bitwise reproducible).  An empty cluster, offsets that decrease or pass n_members, or
 * a member outside [0, Nq) latches SGQ_EINDEX (that cluster's fbar = NaN); a non-finite
 * energy
 * SGQ_ENONFINITE; both are read with sgq_plan_status.  Asynchronous on `stream`. */
int sgq_cluster_energy(sgq_plan* plan, const double* e_node, const int64_t* member_offset,
                       const int32_t* member_node, int64_t n_members, int32_t n_esp,
                       const double* esp_weight, double* fbar, double* energy, void* stream);

/* Predictor + corrector reconstruction on the fine grid (Eq. eq:pc, with the correctors
 * interpolated from the ESPs by linear finite-element shape functions, Eq.
 * phi_approx_scheme).  A mesh object holds a tetrahedral mesh over ESPs that sit on grid
 * points, and, for every point of the grid (the fine grid), the tetrahedron holding it.
 *
 * sgq_fe_mesh_create: HOST arrays; synchronous; uses the current device.
 *   n [3]               grid extents, each in [1, 65536], product < 2^31
 *   esp_center [n_esp]  int64  linear grid index of each ESP; its integer grid coordinates
 *                       (unwrapped: the mesh lives in the box [0, n-1]^3) are the vertex
 *   tets [n_tets*4]     int32  ESP indices of each tetrahedron (any orientation); the
 *                       tetrahedra should tile a region without overlap (a Delaunay
 *                       tetrahedralisation does); zero-volume tetrahedra are ignored
 *   max_fields          1..4: the most fields one sgq_fe_reconstruct call may carry
 * A grid point lies in a tetrahedron when each barycentric coordinate is >= 0 (faces,
 * edges and vertices included), decided exactly (integer volumes).  Each point takes the
 * lowest-numbered tetrahedron that holds it, or none.  Returns SGQ_EINVAL for a bad
 * argument (a vertex index out of range, an ESP outside the grid, ...), SGQ_EHIP when a
 * device call fails.
 *
 * sgq_fe_reconstruct: fields f = 0..n_fields-1, device arrays, asynchronous on `stream`:
 *   esp_values [n_fields][n_esp] double  the full field value f_q at each ESP (e.g. the
 *                                        rho_quadrature density of a plan on the ESPs)
 *   predictor  [n_fields][npts]  double  the predictor f0 on the grid ([z][y][x])
 *   out        [n_fields][npts]  double  f_p = f0_p + sum_i lambda_i (f_{v_i} - f0(r_{v_i}))
 *                                        over the vertices v_i of the point's tetrahedron
 *                                        (lambda its barycentric coordinates); points in no
 *                                        tetrahedron get f0_p; out must not alias the inputs
 * Non-finite inputs propagate to the outputs they touch.  Calls on one mesh must be
 * serialised (they share its corrector scratch).
 *
 * sgq_fe_mesh_location: copies the tetrahedron of every grid point (int32 [npts], -1 for
 * none) into the device array loc, asynchronously on `stream`.
 * sgq_fe_mesh_info: info [5] host int64 out: npts, n_esp, n_tets, kept (non-zero-volume)
 * tetrahedra, bucket edge of the location search. */
typedef struct sgq_fe_mesh sgq_fe_mesh;
int sgq_fe_mesh_create(const int32_t n[3], const int64_t* esp_center, int32_t n_esp,
                       const int32_t* tets, int32_t n_tets, int32_t max_fields,
                       sgq_fe_mesh** out);
int sgq_fe_mesh_destroy(sgq_fe_mesh* mesh);
int sgq_fe_reconstruct(sgq_fe_mesh* mesh, int32_t n_fields, const double* esp_values,
                       const double* predictor, double* out, void* stream);
int sgq_fe_mesh_location(sgq_fe_mesh* mesh, int32_t* loc, void* stream);
int sgq_fe_mesh_info(const sgq_fe_mesh* mesh, int64_t* info);

/* Self-consistency ingredients of the potential in the Hamiltonian (Eq. Eqn:Hamiltonian).
 *
 * sgq_lda_xc: the LDA exchange-correlation energy per volume and potential (Eq. eq:xc),
 *   e_xc = -3/4 (3/pi)^(1/3) rho^(4/3) + rho eps_c(rho) with the Perdew-Wang (1992)
 *   correlation eps_c, and u = d e_xc / d rho; both zero where rho <= 0.  Device arrays of
 *   n doubles: rho in, exc out (optional), vxc out.  Asynchronous on `stream`.
 *
 * sgq_potential_create: a periodic Poisson solver for the grid n (each extent in [1, 1024]
 *   and a product of 2, 3 and 5; fewer than 2^31 points) and spacing h; holds a complex
 *   workspace of m ny nz values of 16 bytes, m = nx/2 + 1 rounded up to a multiple of 8
 *   (whole 128-byte rows).  Uses the current device.
 * sgq_poisson: phi with -(1/4 pi) L phi = s - mean(s) and mean(phi) = 0 (Eq. eq:poisson),
 *   L the sixth-order FD Laplacian of the Hamiltonian on the periodic grid, solved exactly
 *   for that operator by FFT.  Device arrays [nz][ny][nx] double: source in, phi out;
 *   mean [1] out (optional): mean(s), the uniform part the periodic problem cannot hold.
 * sgq_effective_potential: from the electron density rho and the nuclear charge density b
 *   (optional, NULL = 0): v = phi[rho + b] + u(rho); phi, exc and mean are optional outputs
 *   as above.  One FFT pass sequence with the exchange-correlation term fused into its last
 *   pass.
 * Outputs must not alias inputs.  Calls on one solver must be serialised (they share its
 * workspace); all are asynchronous on `stream`. */
typedef struct sgq_potential sgq_potential;
int sgq_lda_xc(const double* rho, int64_t n, double* exc, double* vxc, void* stream);
int sgq_potential_create(const int32_t n[3], double h, sgq_potential** out);
int sgq_potential_destroy(sgq_potential* pot);
int sgq_poisson(sgq_potential* pot, const double* source, double* phi, double* mean,
                void* stream);
int sgq_effective_potential(sgq_potential* pot, const double* rho, const double* b, double* v,
                            double* phi, double* exc, double* mean, void* stream);

/* Retained forward bases (checkpointed Lanczos vectors for the adjoint, Eq. eq:free_cg).
 * With enable != 0 the plan allocates storage for the Lanczos basis and the u_j = H q_j
 * rows of R nodes, 2 K_max n_pad values of the storage precision per node (17.2 MB for
 * 33^3 points at K = 60 in FP32; 141 GB for 8192 such nodes).  max_bytes = 0 retains every
 * node (R = Nq); max_bytes > 0 retains the R = min(Nq, max_bytes / per-node bytes) nodes
 * that are costliest to recompute, n (3K + K(K+1)/2) from the front of the plan's queue.
 * rho_quadrature / band_energy then write those nodes' rows there.  The next
 * band_energy_backward call with the same v_loc, atom_R and proj_E pointers takes the
 * retained rows of those nodes instead of recomputing their forward Lanczos and recomputes
 * the others; both calls hash the contents of those inputs on the device (64-bit, order
 * independent), and when the hashes differ (inputs overwritten in place in between) the
 * backward recomputes every node.  The result is bitwise the full recompute's when the
 * forward ran each node with the backward's lanes for it (512 for FP32 cubes of 37 to 49
 * points, 256 for the others); after another autotuned shape the retained rows differ
 * from a recompute by rounding only.  The backward consumes them (it overwrites the
 * u_j rows), and any other call that runs a forward launch (sgq_plan_autotune, the plain
 * schedule) invalidates them; an invalid or mismatched retention falls back to the
 * recompute.  Every call first waits for the device and frees the storage a
 * previous call allocated; enable = 0 stops there.  n_retained [1] (optional, host) receives
 * R.  Returns SGQ_EINVAL for a null plan, max_bytes < 0, or a max_bytes below one node's
 * rows; SGQ_ENOMEM when the storage does not fit (retention is then off). */
int sgq_plan_set_retain(sgq_plan* plan, int enable, int64_t max_bytes, int64_t* n_retained);

/* Launch capture.  With enable != 0 (the default), rho_quadrature and band_energy on a
 * stream other than the legacy default stream capture their launch sequence (setup
 * kernels, the persistent Lanczos-Gauss kernel, the weighted sum) into a HIP graph on the
 * first call and replay it while the pointers, mu, kT, integrand and launch shape are
 * unchanged; any change re-captures.  The sequence contains kernels only.  Calls on the
 * default stream, or on a stream the caller is already capturing, launch directly.
 * enable = 0 always launches directly.  Returns SGQ_EINVAL for a null plan. */
int sgq_plan_set_graph(sgq_plan* plan, int enable);

/* Launch-shape autotuner.  Times the candidate shapes of the persistent forward kernel
 * (lanes per node: 128, 256 or 512; resident workgroups per CU: 1 to 3; FP64 plans use 256
 * lanes) on `sample_nodes` nodes drawn evenly from the plan's cost-sorted node list, with
 * the given inputs (same meaning as rho_quadrature), and keeps the fastest for the plan:
 * three timed rounds over all candidates after a warm-up round, each candidate's best
 * round counting, and the default shape (256 lanes, two workgroups per CU) kept unless
 * another is more than 1 % faster.  The choice is cached per problem shape (device, precision, cube size, depth, projector
 * box) for the process and, when the environment variable SGQ_TUNE_CACHE names a file,
 * appended to that file and read from it by later processes.  May grow the plan's
 * workspace (SGQ_ENOMEM if that fails).  Synchronous on `stream`.
 *   chosen [2] int32  out (optional, host): lanes per node, workgroups per CU       */
int sgq_plan_autotune(sgq_plan* plan, const double* v_loc, const double* atom_R,
                      const double* proj_E, double mu, double kT, int sample_nodes,
                      void* stream, int32_t* chosen);

/* Wait for the plan's last call and report a latched device-side error (SGQ_OK,
 * SGQ_ENONFINITE, SGQ_ELIMIT, SGQ_ERANGE or SGQ_EINDEX); the latch is cleared by the
 * next compute call. */
int sgq_plan_status(sgq_plan* plan, int32_t* host_status);

/* Message of the last error raised on the calling thread ("" if none). */
const char* sgq_last_error(void);

/* Host-only Gauss rule of a symmetric tridiagonal (the same QR sweeps the kernels run):
 *   alpha [K], beta [K-1] host arrays; theta [K] out ascending, weight [K] out = squared
 *   first eigenvector components.  For testing the eigensolver on a CPU. */
int sgq_gauss_rule_host(const double* alpha, const double* beta, int K, double* theta,
                        double* weight);

/* Validate a problem and node arrays without touching the GPU (no plan is made). */
int sgq_validate(const sgq_problem* prob, const int64_t* center, const int32_t* half_width,
                 const int32_t* depth);

#ifdef __cplusplus
}
#endif

#endif /* SGQ_H */
