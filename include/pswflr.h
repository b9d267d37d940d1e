/*
 * pswflr.h -- C ABI of the MI355X (gfx950) PSWF-LR reciprocal-space path.
 *
 * What is computed (arXiv 2606.06617, Eq. Fourier and Methods,
 * "Accelerating atom-grid spreading with PSWFs"): for each inverse-power
 * channel c with exponent p_c in {1..6} and per-atom latent variables
 * q_i^(c), the truncated Fourier-space energy
 *
 *   E_k^(c) = 1/(2V) sum_{0 < |k| <= k_c} Phi_p(|k|) |sum_i q_i exp(i k.r_i)|^2
 *
 * evaluated by the four-step mesh algorithm (PSWF spreading onto a periodic
 * grid, batched 3D FFT, diagonal scaling by Phi_p / What^2, reduction), plus
 * its exact adjoint (inverse FFT and gather) for potentials dE/dq_i and
 * forces F_i = -dE/dr_i, and the virial.  Phi_p is the Fourier transform of
 * the PSWF-mollified kernel G_p(r)/r^p (Eq. PhiH), k_c = c / r_c (Methods,
 * "Parameter selection").  The zero-frequency term E_0 (Eqs. Correction,
 * Correction3r) and the self term E_self (Methods, "Implementation
 * details") are returned separately per channel, followed by the long-range
 * energy of the MLIP decomposition, E_lr = sum_c (E_k + E_0) (Eq. Fourier);
 * the complete split of Eq. realLR is E_real + E_lr - sum_c E_self.
 *
 * Conventions
 *  - Units: lengths in the caller's unit (Angstrom in the paper); energies in
 *    q^2 / length^p; any Coulomb or C6 prefactor is applied by the caller.
 *  - Cell: the cell tensor of the Fig. 1 caption, a 3x3 matrix H whose rows
 *    are the lattice vectors (pswflr_params.cell), or an orthorhombic box
 *    H = diag(box) when cell is all zeros; origin at 0.  The grid axes run
 *    along the lattice vectors (M_a points on a_a), wave vectors are
 *    k = 2 pi H^-1 m, V = |det H|.  Positions outside the cell are wrapped
 *    (periodically, through their fractional coordinates).
 *  - Memory: every array argument of the execute calls is a DEVICE pointer
 *    owned by the caller; the library never allocates in the execute calls.
 *    A plan owns a small device table (kilobytes) allocated at creation.
 *  - Streams: work is enqueued on the given hipStream_t (NULL = the null
 *    stream) and is asynchronous; outputs are valid once the stream has
 *    reached that point.  A plan may be used concurrently on several
 *    streams as long as each call has its own workspace.
 *  - Errors: argument errors are detected on the host before any launch and
 *    returned as a status; no exception crosses the ABI.  Launch failures are
 *    returned as PSWFLR_ERR_DEVICE.  pswflr_last_error() gives the message of
 *    the last failure on the calling thread.  Values on the device are not
 *    inspected unless the plan has PSWFLR_FLAG_CHECK_INPUTS; without it a
 *    non-finite position makes E_lr, every E_k and the virial NaN (the atom
 *    itself is placed at the origin so that every kernel stays in bounds)
 *    and non-finite charges propagate into the sums.
 */
#ifndef PSWFLR_H
#define PSWFLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSWFLR_MAX_CHANNELS 64
#define PSWFLR_MAX_SUPPORT 8
#define PSWFLR_MAX_GRID 1024

/* Plan flags (pswflr_params.flags).
 * PSWFLR_FLAG_CHECK_INPUTS: every execute call first checks on the device
 * that all positions and charges are finite and waits for the answer; a
 * non-finite value returns PSWFLR_ERR_INVALID_ARG and nothing else runs.
 * The wait makes the call synchronous: meant for debugging and for callers
 * that take inputs from untrusted sources. */
#define PSWFLR_FLAG_CHECK_INPUTS 1u

typedef struct pswflr_plan_s *pswflr_plan; /* opaque, immutable after create */
typedef void *pswflr_stream;               /* a hipStream_t */

typedef enum {
  PSWFLR_OK = 0,
  PSWFLR_ERR_INVALID_ARG = 1, /* a value out of range or a NULL pointer    */
  PSWFLR_ERR_UNSUPPORTED = 2, /* valid but not implemented (grid factors)  */
  PSWFLR_ERR_WORKSPACE = 3,   /* workspace missing or too small            */
  PSWFLR_ERR_DEVICE = 4,      /* a HIP call or kernel launch failed        */
  PSWFLR_ERR_OOM = 5,         /* plan table allocation failed              */
  PSWFLR_ERR_INTERNAL = 6
} pswflr_status;

/* Plan parameters (Methods, "Parameter selection").  Fields left at 0 (or
 * <= 0 for doubles) are chosen automatically from `tol`. */
typedef struct {
  int32_t n_channels;                /* C, 1..PSWFLR_MAX_CHANNELS             */
  int32_t p[PSWFLR_MAX_CHANNELS];    /* exponent of channel c, 1..6           */
  double box[3];                     /* orthorhombic edges, > 0               */
  double r_c;                        /* short-range cutoff, > 0               */
  double c;                          /* mollifier bandwidth; <= 0: ln(3/tol)  */
  double tol;                        /* target relative tolerance, (0, 0.1]   */
  int32_t grid[3];                   /* M_x, M_y, M_z; 0: from tol. Each must
                                        factor into 2, 3, 5; M_z even;
                                        support <= M <= PSWFLR_MAX_GRID;
                                        M_x M_y M_z < 2^30                   */
  int32_t support;                   /* P points per axis, 2..8; 0: from tol  */
  double c_spread;                   /* window bandwidth; <= 0: minimiser of a
                                        force-weighted aliasing estimate     */
  int32_t tile[3];                   /* binning/spreading tile edges; 0: the
                                        planner's choice.  Each must divide
                                        the grid edge (autotuner knob)       */
  uint32_t flags;                    /* PSWFLR_FLAG_* bits, 0 for none        */
  double cell[9];                    /* general cell: lattice vectors as rows
                                        (row-major H); finite, non-singular
                                        and not degenerate (every width across
                                        a lattice plane > 1e-3 of the vector
                                        lengths).  All zeros: the orthorhombic
                                        box above; otherwise box is ignored.
                                        Automatic grids use |a_a| per axis  */
} pswflr_params;

/* Resolved plan (Methods, "Parameter selection"): what the automatic
 * choices became (c = ln(3 / tol) splits the tolerance in thirds between
 * the band limit, the spreading window and the rest; h <= eta pi / k_c;
 * the smallest P whose aliasing estimate meets tol / 3), and the workspace
 * the caller must provide for up to max_atoms atoms. */
typedef struct {
  double c, r_c, k_c, c_spread, eta;
  double h[3];
  double volume;
  int32_t grid[3];
  int32_t support;
  int32_t n_channels;
  int32_t kz_keep;        /* half-spectrum z columns kept (|k_z| <= k_c)    */
  int32_t ny_keep;        /* y frequencies kept after the y transform        */
  int32_t tile[3];        /* spreading/gather tile edge (grid points)        */
  int32_t cg_spread;      /* channels per spreading launch                   */
  int32_t cg_gather;      /* channels per LDS pass of the gather             */
  int64_t xcols;          /* (k_y, k_z) columns the fused x pass transforms  */
  int64_t max_atoms;
  size_t workspace_bytes; /* bytes needed by pswflr_execute                  */
  size_t grid_offset;     /* byte offset of the real grids [C][Mx][My][Mz]   */
  double self_coef[PSWFLR_MAX_CHANNELS]; /* E_self^(c) = self_coef * sum q^2 */
  double zero_coef[PSWFLR_MAX_CHANNELS]; /* E_0^(c) = zero_coef * (sum q)^2  */
  double cell[9];         /* the cell H in use (rows: lattice vectors)       */
} pswflr_info;

/* Build a plan: host FP64 set-up of the PSWF, the kernel and window
 * polynomial tables, the FFT factorisation and the workspace layout; copies
 * a few kilobytes of tables to the current device.  max_atoms bounds the
 * atom count of every later execute call.
 * Errors: INVALID_ARG (NULL, ranges above), UNSUPPORTED (grid not 2,3,5-
 * smooth or odd M_z), OOM, DEVICE. */
pswflr_status pswflr_plan_create(const pswflr_params *params, int64_t max_atoms,
                                 pswflr_plan *out);

/* Copy the resolved parameters and sizes (Methods, "Parameter selection")
 * into *out, a caller-owned struct.  Errors: INVALID_ARG (NULL). */
pswflr_status pswflr_plan_info(pswflr_plan plan, pswflr_info *out);

/* Release the plan (the tables of Methods, "Parameter selection").  Its
 * device table goes back to a per-process pool (no
 * device-wide wait) and is handed to a later plan only once the event
 * recorded at the end of this plan's last call has completed; a plan used
 * on several streams at once must have those streams synchronised by the
 * caller first.  Never blocks. */
pswflr_status pswflr_plan_destroy(pswflr_plan plan);

/* One evaluation (the whole hot path: the four steps after Eq. EthetaLR in
 * Methods, "Accelerating atom-grid spreading with PSWFs", and their adjoint
 * for forces, Fig. 1 caption) on `stream`.
 *   pos       [N][3] float, positions (wrapped into the cell)
 *   q         [C][N] float, latent variables per channel (SoA)
 *   energy    [3C + 1] double (required): per channel E_k, E_0, E_self,
 *             then E_lr = sum_c (E_k + E_0) summed in channel order
 *   forces    [N][3] float or NULL: F_i = -d(sum_c E_k + E_0)/dr_i
 *   virial    [6] double or NULL: W = -dE/d(strain) of sum_c (E_k + E_0),
 *             order xx, yy, zz, xy, xz, yz
 *   potential [C][N] float or NULL: d(E_k + E_0)/dq_i^(c)
 * When forces and potential are both NULL only the forward transforms run
 * (the energy needs no inverse FFT); the spectrum is then left in the
 * workspace for pswflr_backward.
 * workspace: device memory of at least info.workspace_bytes, 256-byte
 * aligned, not shared with concurrent calls.  0 <= N <= max_atoms.
 * Errors: INVALID_ARG, WORKSPACE, DEVICE. */
pswflr_status pswflr_execute(pswflr_plan plan, pswflr_stream stream, void *workspace,
                             size_t ws_bytes, int64_t n_atoms, const float *pos,
                             const float *q, double *energy, float *forces,
                             double *virial, float *potential);

/* Second derivatives for force-matching training (Fig. 1 caption: forces
 * are gradients of the energy, so a loss on forces needs the derivatives of
 * the forces).  Given v [N][3] (device float, dL/dF_i of a loss L on the
 * forces of the immediately preceding pswflr_execute, which must have
 * computed forces or potentials with this plan, workspace, positions and
 * charges, and no other call on that workspace in between), writes the
 * derivatives of L through the forces:
 *   grad_q   [C][N] float: dL/dq_i^(c) = -v_i . grad phi_c(r_i) - (W^T A u_c)_i
 *   grad_pos [N][3] float: dL/dr_i = -sum_c q_i^(c) (Hess phi_c(r_i) v_i
 *                                    + grad_i (W^T A u_c))
 * with phi_c the forward's potential, u_c the dipole grid sum_i q_i^(c)
 * (v_i . grad_{r_i}) W(n h - r_i), W the PSWF window and A the forward's
 * convolution (Eq. EthetaLR).  Both outputs are required (device, caller-
 * owned).  The forward's potential grid in the workspace is consumed.
 * Errors: INVALID_ARG, WORKSPACE, DEVICE. */
pswflr_status pswflr_force_vjp(pswflr_plan plan, pswflr_stream stream, void *workspace,
                                size_t ws_bytes, int64_t n_atoms, const float *pos,
                                const float *q, const float *v, float *grad_q, float *grad_pos);

/* The real-space complement of the split (Eq. realLR; Methods,
 * "Implementation details"): for each channel c,
 *   E_real^(c) = 1/2 sum_n sum'_{i,j} q_i q_j (1 - G_p(r)) / r^p,
 * r = |r_j - r_i + n H| < r_c over all periodic images n (the prime drops
 * i = j at n = 0), with G_p the PSWF mollifier of Eqs. G1, G6, G at the
 * plan's c and r_c.  Together with pswflr_execute this gives the complete
 * energy of Eq. realLR: E = sum_c (E_real + E_k + E_0 - E_self).
 *   energy    [C] double (required): E_real per channel
 *   forces    [N][3] float or NULL: -dE_real/dr_i summed over channels
 *   virial    [6] double or NULL: -dE_real/d(strain), order as execute
 *   potential [C][N] float or NULL: dE_real/dq_i^(c)
 * Same plan, workspace (its real-space part: an execute's results in the
 * same workspace, spectrum included, are left intact), stream semantics and
 * errors as pswflr_execute.  Pairs at zero distance are skipped. */
pswflr_status pswflr_realspace(pswflr_plan plan, pswflr_stream stream, void *workspace,
                               size_t ws_bytes, int64_t n_atoms, const float *pos,
                               const float *q, double *energy, float *forces,
                               double *virial, float *potential);

/* pswflr_execute without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments and results as
 * pswflr_execute minus the workspace: the library's own scratch array of
 * 64 MiB per device (reserved when the library is loaded, held until the
 * process ends) takes its place.  Nothing is allocated: no hipMalloc,
 * hipFree, event or pinned buffer, no timing events even while profiling
 * is on.  Limits and rules:
 *  - the plan's workspace (pswflr_info.workspace_bytes, set by its
 *    max_atoms) must fit the 64 MiB, else PSWFLR_ERR_WORKSPACE;
 *  - plans with PSWFLR_FLAG_CHECK_INPUTS are refused (INVALID_ARG): the
 *    check waits on the host;
 *  - every call on one device shares that device's scratch, which keeps
 *    the last call's contents: calls that overlap on one device (two
 *    streams, or two threads) race and give wrong results; serialise them;
 *  - the call does not record the plan's last-use event: synchronise the
 *    stream before destroying the plan.
 * Errors: INVALID_ARG, WORKSPACE, DEVICE. */
pswflr_status pswflr_execute_noalloc(pswflr_plan plan, pswflr_stream stream, int64_t n_atoms,
                                     const float *pos, const float *q, double *energy,
                                     float *forces, double *virial, float *potential);

/* Adjoint of an energy-only pswflr_execute (same plan, workspace, positions
 * and charges, no other call on that workspace in between): given
 * grad_energy [C] (device double, dL/dE_c where E_c = E_k + E_0 of channel
 * c), writes dL/dq [C][N] and dL/dr [N][3] (either may be NULL; device
 * float, caller-owned).  This is the hand-written backward of the
 * differentiable energy (Fig. 1 caption: forces and charge gradients by
 * differentiation of Eq. Fourier): the spectrum scaled by Phi_p / What^2
 * (Eq. EthetaLR), the inverse transforms and the gather with the window
 * and its gradient.  Errors: INVALID_ARG, WORKSPACE, DEVICE. */
pswflr_status pswflr_backward(pswflr_plan plan, pswflr_stream stream, void *workspace,
                              size_t ws_bytes, int64_t n_atoms, const float *pos,
                              const float *q, const double *grad_energy,
                              float *grad_q, float *grad_pos);

/* Derivative of the energy with respect to the cell tensor (Fig. 1
 * caption: the cell is an input and the virial comes from differentiation;
 * constant-pressure dynamics moves the cell).  From a virial W [6] (device
 * double, xx, yy, zz, xy, xz, yz, as written by pswflr_execute or
 * pswflr_realspace with this plan: W = -dE/d(strain), positions moving with
 * the cell), writes
 *   grad_cell [9] device double, row-major: dE/dH_ab = -(H^-T W)_ab
 * the derivative at fixed fractional coordinates (H -> H (1 + e)^T moves
 * every position r -> (1 + e) r).  One work-item on `stream`; both pointers
 * caller-owned.  Errors: INVALID_ARG, DEVICE. */
pswflr_status pswflr_cell_gradient(pswflr_plan plan, pswflr_stream stream, const double *virial,
                                   double *grad_cell);

/* Many structures in one call (MLIP training batches, serving mixes; the
 * paper evaluates configurations of many sizes and boxes, Methods,
 * "Performance comparison in differentiable long-range evaluations").  Each
 * entry has its own plan (box, grid and channels may differ) and its own
 * device pointers; semantics per entry are those of pswflr_execute.  Each
 * stage is one launch covering every entry (a device table maps a block to
 * its entry); entries with more than 12 channels are evaluated one call at
 * a time instead.  Results for an entry do not depend on the other entries.
 * The workspace (pswflr_batch_workspace gives its size) holds a header and
 * one per-entry workspace; it is owned by the caller and must not be used by
 * another call until this one has completed on the stream. */
typedef struct {
  int64_t n_atoms;
  const float *pos;
  const float *q;
  double *energy;
  float *forces;
  double *virial;
  float *potential;
} pswflr_io;

/* Bytes of workspace pswflr_execute_batch needs for these plans and atom
 * counts (host arrays of n entries).  Errors: INVALID_ARG. */
pswflr_status pswflr_batch_workspace(int32_t n, const pswflr_plan *plans,
                                     const int64_t *n_atoms, size_t *bytes);
pswflr_status pswflr_execute_batch(int32_t n, const pswflr_plan *plans,
                                   const pswflr_io *io, pswflr_stream stream,
                                   void *workspace, size_t ws_bytes);

/* The batched call with every array flat: the structures' atoms, charges
 * and outputs follow each other in one device array each, in batch order.
 *   n_atoms   [n] host: atoms of each structure (N_i)
 *   pos       [sum N_i][3]; q: the blocks [C_i][N_i] one after another
 *   energy    the blocks [3 C_i + 1]; forces [sum N_i][3] or NULL;
 *   virial    [n][6] or NULL; potential: blocks [C_i][N_i] or NULL
 * Same semantics, workspace (pswflr_batch_workspace) and errors as
 * pswflr_execute_batch; the per-structure pointers are formed here, so the
 * caller passes four pointers instead of a table. */
pswflr_status pswflr_execute_batch_flat(int32_t n, const pswflr_plan *plans, const int64_t *n_atoms,
                                        const float *pos, const float *q, double *energy,
                                        float *forces, double *virial, float *potential,
                                        pswflr_stream stream, void *workspace, size_t ws_bytes);

/* Adjoint of an energy-only batched forward (pswflr_execute_batch or
 * _flat with forces and potentials NULL, same plans, atoms, workspace, and
 * no other call on that workspace in between): the hand-written backward of
 * every structure's energy at once (Fig. 1 caption: gradients by
 * differentiation; the scaled inverse transforms and the gather, one launch
 * per stage over all structures).
 *   grad_energy [sum C_i] device: dL/dE_c of each structure's channels
 *   grad_q      blocks [C_i][N_i] or NULL: dL/dq
 *   grad_pos    [sum N_i][3] or NULL: dL/dr
 * Errors: INVALID_ARG, WORKSPACE, DEVICE. */
pswflr_status pswflr_backward_batch_flat(int32_t n, const pswflr_plan *plans, const int64_t *n_atoms,
                                         const float *pos, const float *q, const double *grad_energy,
                                         float *grad_q, float *grad_pos, pswflr_stream stream,
                                         void *workspace, size_t ws_bytes);

/* Per-stage device timing, for measurement (the paper times whole
 * forward+backward evaluations after warm-ups; Methods, "Performance
 * comparison in differentiable long-range evaluations").  While enabled,
 * every stage launch of the execute calls is bracketed by a pair of
 * hipEvents on the caller's stream.  pswflr_profile_read waits for the
 * recorded events, writes per-stage total milliseconds and launch counts
 * ([PSWFLR_NUM_STAGES] each) and forgets them.  Not for concurrent use of
 * one plan from several threads while enabled. */
enum {
  PSWFLR_STAGE_SORT = 0,       /* binning, cell order                      */
  PSWFLR_STAGE_QSUM = 1,       /* per-channel sum q, sum q^2 (launched with
                                  the sort and timed as its part)         */
  PSWFLR_STAGE_SPREAD = 2,     /* step (i), one launch per channel group   */
  PSWFLR_STAGE_FFT_Z = 3,      /* z real-to-complex                        */
  PSWFLR_STAGE_FFT_Y = 4,      /* y forward                                */
  PSWFLR_STAGE_FFT_X_SCALE = 5,/* x forward, scaling, reduction, x inverse */
  PSWFLR_STAGE_REDUCE = 6,     /* FP64 energy and virial                   */
  PSWFLR_STAGE_IFFT_Y = 7,
  PSWFLR_STAGE_IFFT_Z = 8,
  PSWFLR_STAGE_GATHER = 9,
  PSWFLR_NUM_STAGES = 10
};
pswflr_status pswflr_profile_enable(pswflr_plan plan, int enable);
/* As pswflr_profile_enable, restricted to the stages whose bit
 * (1u << PSWFLR_STAGE_*) is set in stage_mask; 0 turns timing off, and
 * pswflr_profile_enable(plan, 1) is the mask of every stage.  The other
 * launches then carry no event records, so one stage can be timed inside a
 * throughput measurement without slowing the rest.
 * Errors: INVALID_ARG (NULL plan, a bit above the last stage). */
pswflr_status pswflr_profile_stages(pswflr_plan plan, uint32_t stage_mask);
pswflr_status pswflr_profile_read(pswflr_plan plan, double *ms_total, int64_t *launches);

/* Static text naming a status (not a passage of the paper: error
 * reporting of this interface). */
const char *pswflr_status_string(pswflr_status status);
/* Copies the last error message of the calling thread (NUL-terminated,
 * truncated to len bytes) into the caller's buffer. */
void pswflr_last_error(char *buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* PSWFLR_H */
