/*
 * dgmax.h -- C-ABI of the MI355X discontinuous Galerkin Maxwell curl engine.
 *
 * The library applies the central-flux DG curl operator of the loss-free
 * time-domain Maxwell equations on affine tetrahedra (Koutschan, Lehrenfeld,
 * Schoeberl, arxiv 1104.4208):
 *     eps dE/dt =  curl H,   mu dH/dt = -curl E                  (Section 2)
 * discretised with piecewise polynomials of degree p in an L2-orthonormal
 * Dubiner basis (Sections 3.1 and 4.2.2), the covariant map (Section 3.2.1),
 * element-local mass inverses (Section 3.3.1; for material linear inside the
 * elements the approximate inverse of Section 3.3.2) and the central flux
 * (Section 2.1, eq. semidiscrete), advanced by symplectic Euler / leapfrog
 * with H updated first (Section 3).
 *
 * Conventions shared by every entry point
 *  - Every function returns an int status: DGM_OK (0) or a negative DGM_ERR_*
 *    code; dgm_last_error() then returns a thread-local message.  No C++
 *    exception crosses this interface.
 *  - Field arrays (E, H, dE, dH, H_next) are caller-owned DEVICE buffers
 *    shaped (3, N, K), contiguous, element index fastest, of type float
 *    (dtype DGM_F32) or double (DGM_F64), with N = dgm_num_modes(p) and K the
 *    number of tetrahedra.  Entry [c][m][e] is component c of the reference
 *    covariant coefficient of volume mode m on element e: the physical field
 *    on e is F_e^{-T} sum_m Ehat_m phi_m(xhat), where F_e = [v1-v0, v2-v0,
 *    v3-v0] is built from the element's vertices sorted by ascending global
 *    id, and the mode order is the one reported by dgm_mode_index.
 *  - Work is enqueued on the caller's HIP stream; calls that return host
 *    values (dgm_energy, dgm_estimate_dt) synchronise that stream.
 *  - The library never frees caller memory.  It owns the mesh handle and the
 *    device arrays it allocates for it (geometry, neighbour codes, scratch).
 *  - Walls: every face without a neighbour is a perfect electric conductor
 *    (ghost states E_nb = -E, H_nb = H).
 *  - Calls on one mesh handle must not overlap in time (they share scratch).
 */
#ifndef DGMAX_H
#define DGMAX_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dgm_mesh dgm_mesh;

enum { DGM_F32 = 0, DGM_F64 = 1 };
/* 16-bit operand precisions of the dense matrix-core variant (FP32 accumulation). */
enum { DGM_BF16 = 2, DGM_F16 = 3 };

enum {
  DGM_OK = 0,
  DGM_ERR_ARG = -1,              /* null pointer, bad size, order out of range */
  DGM_ERR_MESH_DEGENERATE = -2,  /* |det F| < 1e-12 h^3 or repeated vertex */
  DGM_ERR_MESH_NONMANIFOLD = -3, /* a face shared by more than two tetrahedra */
  DGM_ERR_MATERIAL = -4,         /* eps or mu not strictly positive / not finite */
  DGM_ERR_OOM = -5,              /* device allocation failed */
  DGM_ERR_HIP = -6,              /* a HIP runtime call failed (message has the HIP error) */
  DGM_ERR_UNSTABLE = -7,         /* non-finite energy or state detected */
  DGM_ERR_STATE = -8             /* order not set, or a batch call out of sequence */
};

/* Thread-local description of the last error returned on this thread. */
const char* dgm_last_error(void);

/* Number of volume modes (p+1)(p+2)(p+3)/6 and face modes (p+1)(p+2)/2. */
int dgm_num_modes(int p);
int dgm_num_face_modes(int p);
/* Highest order compiled into this library for dtype (DGM_F32 / DGM_F64). */
int dgm_max_order(int dtype);

/* Mode m (0 <= m < N) of order p is phi_{i,j,k} of Section 4.2.2 scaled to unit
 * norm: i indexes the innermost (z) Legendre factor, j the y factor, k the x
 * factor.  Modes are ordered by total degree, then i, then j. */
int dgm_mode_index(int p, int m, int* i, int* j, int* k);

/* Build a mesh from host arrays (copied): verts[nv][3] (FP64), tets[nt][4]
 * (vertex ids in [0, nv)).  Vertices of each tetrahedron are sorted by
 * ascending id, so both sides of a face parametrise it identically; the
 * neighbour map is built from shared vertex triples (Section 3, locality of
 * the DG curl).  1 <= nt <= 2^28 - 64 (an empty mesh is DGM_ERR_ARG).  Errors: DGM_ERR_ARG, DGM_ERR_MESH_DEGENERATE,
 * DGM_ERR_MESH_NONMANIFOLD, DGM_ERR_OOM, DGM_ERR_HIP.  Material defaults to
 * eps = mu = 1 and the order must be set before any field operation. */
int dgm_create_mesh(const double* verts, int64_t nv, const int64_t* tets, int64_t nt, dgm_mesh** out);

/* Release the handle and every device array the library allocated for it. */
int dgm_destroy(dgm_mesh* mesh);

/* Number of tetrahedra of the mesh. */
int dgm_num_elements(const dgm_mesh* mesh, int64_t* K);

/* Select the polynomial order p (1 <= p <= dgm_max_order(dtype) at use time). */
int dgm_set_order(dgm_mesh* mesh, int p);

/* Per-element piecewise-constant permittivity and permeability (host arrays of
 * length K, each > 0; NULL means 1).  Folds the flat-element mass inverse
 * |det F| eps F^{-1} F^{-T} (Section 3.3.1, eq. massintegral) into per-element
 * factors.  Every value is checked before anything is uploaded, so a rejected
 * call leaves the mesh's previous material in place.  Errors: DGM_ERR_MATERIAL,
 * DGM_ERR_HIP. */
int dgm_set_material(dgm_mesh* mesh, const double* eps, const double* mu);

/* Permittivity and permeability that vary linearly inside every element (Section
 * 3.3.2): host arrays (K,4) row-major, the values at the element's four vertices in
 * the order the element was given to dgm_create_mesh (each > 0; NULL means 1), so a
 * field continuous across faces or one that jumps between elements are both
 * possible.  The mass matrix of such a material is no longer the flat one; its
 * inverse is replaced by the approximate inverse of Section 3.3.2: the rate's point
 * values at the collapsed Gauss rule with p + 1 points per direction (the reverse of
 * numerical integration), divided by the material at the points, integrated back,
 *     (P r)_a = sum_x w_x phi_a(x) (sum_b phi_b(x) r_b) / m(x),
 * applied to every component (sum factorisation, O(p^4) per element: one generated
 * kernel per order).  The rule is laid on the element's reference map with vertices
 * sorted by global id.  P is symmetric positive definite and exact for constant
 * material (then this reproduces dgm_set_material up to rounding).  dgm_apply_curl,
 * dgm_step, dgm_step_probe (E mapped by the unit-material factors), dgm_energy
 * (W and Q with M~ = P^{-1}, one preconditioned conjugate-gradient solve per field,
 * in FP64 where the orders have FP64 kernels) and dgm_estimate_dt (in the M~ inner
 * product) use it, with equal or mixed orders; the stabilised flux, the dense variant,
 * batch slots and dgm_step_noalloc return DGM_ERR_STATE until dgm_set_material is
 * called again.  Every value is checked before anything changes.  Errors:
 * DGM_ERR_MATERIAL, DGM_ERR_OOM, DGM_ERR_HIP. */
int dgm_set_material_linear(dgm_mesh* mesh, const double* eps, const double* mu);

/* The approximate mass inverse of dgm_set_material_linear alone (Section 3.3.2): for every
 * component c and element, Y[c] = P X[c] with
 *     (P r)_a = sum_x w_x phi_a(x) (sum_b phi_b(x) r_b) / m(x)
 * on the reference element (the collapsed Gauss rule with p + 1 points per direction, weights
 * summing to 1/6, m = eps for field 0 and mu for field 1, linear from the vertex values).
 * For moments f_a = int_T f phi_a dx of a functional, P (f / |det F|) is the approximate
 * inverse of the material-weighted mass matrix applied to them.  X and Y are device arrays
 * of the field's shape (3, N, K) and dtype (N of that field's order), distinct; P acts on the
 * mode index only, so any per-element frame of the components may be used.  One launch of
 * the generated kernel dgm_mass_p{p}; asynchronous on the stream.  Errors: DGM_ERR_STATE
 * without a linear material, DGM_ERR_ARG for a bad field or aliasing arrays. */
int dgm_apply_mass_inverse(dgm_mesh* mesh, int dtype, int field, const void* X, void* Y, hipStream_t stream);

/* Semi-discrete right-hand side (Section 2.1, eq. semidiscrete):
 *     dE = -M_eps^{-1} C^T H  (= eps^{-1} curl_h H),
 *     dH =  M_mu^{-1} C E     (= -mu^{-1} curl_h E),
 * in the covariant layout above.  Either output may be NULL (then the matching
 * input may be NULL too).  Outputs must not alias inputs. */
int dgm_apply_curl(dgm_mesh* mesh, int dtype, const void* E, const void* H, void* dE, void* dH,
                   hipStream_t stream);

/* Stability check of dgm_step (and dgm_step_probe): with every > 0, after every
 * `every` steps of a call and after its last step, the FP64 sum of squares of both
 * fields is formed (one reduction and a stream synchronisation per check); if it is
 * not finite the call stops there, converts the fields back to the covariant layout
 * and returns DGM_ERR_UNSTABLE.  A leapfrog run grows without bound when dt exceeds
 * 2/sqrt(rho) (Section 3), so this catches a time step above the bound.  every = 0
 * (the default) disables the checks; every < 0 is DGM_ERR_ARG. */
int dgm_set_check_interval(dgm_mesh* mesh, int64_t every);

/* nsteps symplectic Euler steps in place (Section 3):
 *     H <- H + dt M_mu^{-1} C E,   E <- E - dt M_eps^{-1} C^T H.
 * dt is the caller's (see dgm_estimate_dt); nsteps >= 0.  Each half step is one
 * kernel that also writes the tangential face traces of the field it updated
 * (per element and face two tangents over the (p+1)(p+2)/2 face modes, each
 * padded to a multiple of 4) for the neighbours in the next half step; the
 * handle keeps these two buffers (allocated on first use, K rounded up to a
 * multiple of 64, times 8 x the padded face-mode count, values of dtype each).
 * When both fields and both trace buffers together exceed 256 MB (the
 * last-level cache) the kernels give their field accesses the nontemporal hint;
 * the arithmetic, and so the result, is the same either way. */
int dgm_step(dgm_mesh* mesh, int dtype, void* E, void* H, double dt, int64_t nsteps, hipStream_t stream);

/* dgm_step that also records, after each step n (0-based), signal[n] = sum_i w_i S_i,
 * a fixed linear functional of E: S are the library's internal coefficients of E
 * during the run (covariant coefficients mapped by the per-element mass inverse and
 * the derivative frame) and w is a device array of E's shape and dtype.  A generic w
 * (e.g. random) sees every mode, which is what a frequency analysis of the time
 * signal needs (the resonance workload of Section 2.2's numerical example).
 * signal: host array of nsteps doubles; synchronises the stream. */
int dgm_step_probe(dgm_mesh* mesh, int dtype, void* E, void* H, double dt, int64_t nsteps, const void* w,
                   double* signal, hipStream_t stream);

/* dgm_step for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and
 * the same arithmetic (bitwise equal results), but the trace buffers and the reduction
 * buffers of the stability check live in a static device workspace of
 * DGM_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on until the
 * process ends; no hipMalloc, hipFree or allocating library routine is called.  A mesh
 * needs 2 x ceil(K/64) x 64 x 8 x ceil((p+1)(p+2)/8) x 4 values of dtype plus 4 KiB
 * (about 64 MiB holds 37,000 tetrahedra at p = 6 in FP32); larger meshes are rejected
 * with DGM_ERR_ARG before any work.  Every call on one GPU shares that GPU's workspace:
 * calls that overlap in time on one GPU (other threads, other streams) race and must be
 * serialised by the caller.  The workspace needs no clearing (every value is written
 * before it is read).  Other arguments, errors and the check interval as dgm_step. */
#define DGM_NOALLOC_SCRATCH_BYTES (64u << 20)
int dgm_step_noalloc(dgm_mesh* mesh, int dtype, void* E, void* H, double dt, int64_t nsteps, hipStream_t stream);

/* FP64 energies: out[0] = W = 1/2 (E, M_eps E) + 1/2 (H, M_mu H)  (Section 2.1),
 * out[1] = Q = 1/2 (E, M_eps E) + 1/2 (H, M_mu H_next), the quantity the
 * H-first symplectic Euler step conserves exactly.  H_next is the H of the next
 * step; if NULL it is computed internally as H + dt dH(E) (H itself when dt is
 * 0, so Q = W).  The reductions run at any order; forming H_next needs the
 * order compiled for dtype.  Returns DGM_ERR_UNSTABLE if W or Q is not finite
 * (out is still written). */
int dgm_energy(dgm_mesh* mesh, int dtype, const void* E, const void* H, const void* H_next, double dt,
               double out[2], hipStream_t stream);

/* Time step from the stability bound of Section 3: power iteration (iters
 * steps, start vector from SplitMix64(seed) over the (3,N,K) layout, mapped to
 * [-1,1)) estimates rho = rho(M_mu^{-1/2} C M_eps^{-1} C^T M_mu^{-1/2}); the
 * result is dt = cfl * 2 / sqrt(rho) (the printed bound lacks the square root;
 * leapfrog is stable iff dt <= 2/sqrt(rho)).  rho_out may be NULL.  Runs in
 * FP64 on the device where the order is compiled in FP64 (dgm_max_order), in
 * FP32 with FP64 dot products above it; synchronises the stream. */
int dgm_estimate_dt(dgm_mesh* mesh, double cfl, int iters, uint64_t seed, double* dt, double* rho_out,
                    hipStream_t stream);

/* Mixed orders (Section 2): E of degree pE = pH + 1 and H of degree pH, the pairing
 * the paper chooses because all derivatives fall on E and its test functions
 * (pE == pH is dgm_set_order(mesh, pH)).  E-shaped arrays (E, dE, the probe weights)
 * then have N_E = dgm_num_modes(pE) modes per component and H-shaped ones N_H; the
 * curl maps the N_E modes of E into the N_H rows of H and back, with the lift of each
 * field's face traces (degree of that field) into the other's rows.  dgm_apply_curl,
 * dgm_step, dgm_step_probe, dgm_step_noalloc, dgm_energy and dgm_estimate_dt accept
 * mixed orders; the stabilised flux, the dense variant and batch slots need equal
 * orders (DGM_ERR_STATE).  Built for pH = 1 .. max order - 1 (FP64: pE up to the
 * FP64 maximum).  Errors: DGM_ERR_ARG for another pair or one not built. */
int dgm_set_orders(dgm_mesh* mesh, int pE, int pH);
/* The orders set on the mesh (both 0 before dgm_set_order / dgm_set_orders). */
int dgm_orders(const dgm_mesh* mesh, int* pE, int* pH);

/* Stabilised central flux with face unknowns H^F (Section 2.1), the paper's
 * recommended method: it keeps the discrete energy and removes the spurious
 * modes of the central flux.  Besides E and H the state holds, on every face, a
 * tangential field H^F of degree p with
 *     (h_F/alpha) (dH^F/dt, h^F)_F = ([E] x nu, h^F)_F,
 *     (eps dE/dt, e)_T gains (H^F x nu_T, e)_F on each face of T (twice on walls),
 * [E] = E_s - E_nb across the face (2 E on walls, ghost E_nb = -E), alpha =
 * alpha0 p^2, h_F = 3 min |T| / |F| over the face's elements (the smaller height
 * over F).  The paper prints alpha/h as the face mass; its definition
 * H^F = alpha [E] x nu / (i omega h) and its penalty S ~ alpha/h both give the
 * mass h/alpha used here.  The central entry points above are unaffected.
 *
 * dgm_set_stab_alpha sets alpha0 (> 0; DGM_ERR_ARG otherwise); the stabilised
 * calls below return DGM_ERR_STATE until it is called, and rebuild their face data
 * (host FP64, one upload) after an order change.
 *
 * HF: caller-owned device buffer of dgm_num_face_unknowns() = 8 NF K values of the
 * dtype (NF = dgm_num_face_modes(p)), entry ((k NF + m) 4 + f) K + e = the
 * coefficient of face mode m (the orthonormal triangle basis of the face
 * parametrised by its vertices in ascending global id, modes ordered by degree)
 * of H^F . t_k on local face f of element e, where t_1, t_2 are the face's edge
 * vectors from its lowest-id vertex (both sides of a face agree on them).  A face
 * is held by one side: the element with the smaller index (the element itself on
 * a wall); the other side's entries are neither read nor written. */
int dgm_set_stab_alpha(dgm_mesh* mesh, double alpha0);
int dgm_num_face_unknowns(const dgm_mesh* mesh, int64_t* n);
/* Rates: dH = M_mu^{-1} C E (as dgm_apply_curl) and dHF = dH^F/dt from E (held
 * entries only; the others are set to 0), dE from H and HF.  Any output may be NULL;
 * outputs must not alias inputs. */
int dgm_apply_stab(dgm_mesh* mesh, int dtype, const void* E, const void* H, const void* HF, void* dE, void* dH,
                   void* dHF, hipStream_t stream);
/* nsteps symplectic-Euler steps in place: H and H^F from E, then E from H and H^F
 * (Section 3); honours dgm_set_check_interval as dgm_step does. */
int dgm_step_stab(dgm_mesh* mesh, int dtype, void* E, void* H, void* HF, double dt, int64_t nsteps,
                  hipStream_t stream);
/* out[0] = W + 1/2 sum_F (h_F/alpha) (H^F, H^F)_F, out[1] = Q with the face term
 * 1/2 sum_F (h_F/alpha) (H^F, H^F_next)_F, the quantity the stabilised step
 * conserves exactly; H_next and H^F_next are formed internally (dt = 0: Q = W). */
int dgm_energy_stab(dgm_mesh* mesh, int dtype, const void* E, const void* H, const void* HF, double dt,
                    double out[2], hipStream_t stream);
/* dgm_estimate_dt for the stabilised operator: power iteration on
 * E -> -dE(dH(E), dHF(E)) (the face term raises the spectral radius). */
int dgm_estimate_dt_stab(dgm_mesh* mesh, double cfl, int iters, uint64_t seed, double* dt, double* rho_out,
                         hipStream_t stream);

/* Dense reference-operator variant on the matrix cores.  The same semi-discrete
 * operator as dgm_apply_curl / dgm_step, applied as the dense O(N^2) element
 * matrices that Section 3.2 avoids (curl in the derivative frame, four trace
 * tables and their transposes), batched over tiles of 64 elements with prec =
 * DGM_BF16 or DGM_F16 operands and FP32 accumulation (v_mfma_f32_32x32x16).
 * Fields are FP32 (3, N, K) covariant arrays as above; the field update is FP32.
 * Results differ from the FP32 path by the 16-bit rounding of the operands
 * (about 1e-3 relative for BF16, 1e-4 for FP16).  The first call for an order
 * builds the dense operators (host, then a device copy kept in the handle). */
int dgm_apply_curl_dense(dgm_mesh* mesh, int prec, const float* E, const float* H, float* dE, float* dH,
                         hipStream_t stream);
int dgm_step_dense(dgm_mesh* mesh, int prec, float* E, float* H, double dt, int64_t nsteps, hipStream_t stream);

/* Batched serving: many independent solves advance together.  A batch holds
 * slots (mesh handle, caller-owned FP32 E and H, dt, remaining steps).  Each
 * dgm_batch_advance advances every active slot by min(chunk, remaining) steps
 * with one HIP-graph launch whose kernels (one per order and half step) cover
 * all slots of that order; finished slots are converted back to the covariant
 * layout and reported by dgm_batch_take_finished.  Between dgm_batch_add and
 * completion, E and H hold the library's internal stored-frame coefficients
 * and must not be read or written by the caller.  A mesh handle may back at
 * most one active slot and must not be passed to other calls while its slot is
 * active (the slot runs on the handle's trace buffers).  Results are bitwise equal to dgm_step on the same
 * slot alone (same kernels, same per-element arithmetic).  Not part of the
 * paper (its solver runs one mesh on one core); this is the serving layer. */
typedef struct dgm_batch dgm_batch;
int dgm_batch_create(int chunk, dgm_batch** out);
int dgm_batch_destroy(dgm_batch* batch);
int dgm_batch_add(dgm_batch* batch, dgm_mesh* mesh, float* E, float* H, double dt, int64_t nsteps,
                  hipStream_t stream, int64_t* id);
int dgm_batch_num_active(const dgm_batch* batch, int64_t* n);
/* Advances all active slots and synchronises the stream.  When the set of orders
 * in use, the grid capacity or the cache policy changes, the call first re-captures
 * its HIP graph; HIP calls made by other threads of the process meanwhile can make
 * that capture fail (DGM_ERR_HIP), so other threads should not use the GPU during
 * this call. */
int dgm_batch_advance(dgm_batch* batch, hipStream_t stream);
/* dgm_batch_advance in two halves, so the host can work while a chunk runs:
 * dgm_batch_launch enqueues the chunk (and the retirement of the slots it finishes)
 * on the stream and returns; dgm_batch_wait synchronises that stream.  Between the
 * two the caller may set up other meshes but must not launch, take finished ids
 * (DGM_ERR_STATE) or touch the slots' fields.  If dgm_batch_launch fails after the
 * graph was launched, dgm_batch_wait is still required. */
int dgm_batch_launch(dgm_batch* batch, hipStream_t stream);
int dgm_batch_wait(dgm_batch* batch);
/* *yes = 1 when the next launch will re-capture its graph (see dgm_batch_advance):
 * host-only, so a caller can keep other threads off the GPU for just those launches. */
int dgm_batch_needs_capture(const dgm_batch* batch, int* yes);
/* Copies up to cap finished slot ids into ids and removes them from the list. */
int dgm_batch_take_finished(dgm_batch* batch, int64_t* ids, int64_t cap, int64_t* n);

#ifdef __cplusplus
}
#endif

#endif /* DGMAX_H */
