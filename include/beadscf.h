/*
 * beadscf.h - C ABI of the batched direct-SCF energy/force engine for MI355X.
 *
 * The engine computes, for every replica ("bead", "image" or independent
 * cluster) of a batch, the Born-Oppenheimer energy and force at the
 * closed-shell Hartree-Fock level in a Gaussian basis.  This is the per-replica
 * force provider of the paper's replica simulation: the replica layer hands a
 * set of n nuclear configurations to the electronic-structure layer and gets
 * back the BO energy and force of each (Section 2, Fig. 1a), gathered into
 * per-replica arrays (the zero-filled E[n] and F[n][N_atom][3] of Section 2).
 * The SCF thresholds follow Section 3.1 (density threshold 1e-6, integral
 * cutoff 1e-12), and each replica's previous-step orbitals can seed its next
 * SCF (Section 2, reuse of the molecular orbitals kept in memory).
 *
 * Conventions
 *   - Atomic units throughout: bohr, hartree (Eh), Eh/bohr.
 *   - Instance-major arrays; atoms in input order; xyz fastest.
 *   - Matrices are n x n FP64, symmetric, row-major (= column-major).  Basis
 *     order: atoms in input order, shells in basis-file order, Cartesian
 *     components lexicographic (x,y,z; xx,xy,xz,yy,yz,zz), each component
 *     normalised to unit self-overlap.
 *   - Host arrays passed in are copied before the call returns; outputs go
 *     into caller-owned buffers.  With device_ptrs != 0 the pointers are HIP
 *     device memory on the context's device and the work is ordered on the
 *     context's stream.
 *   - Every call returns a bscf_status (BSCF_OK == 0, errors < 0); nothing
 *     throws across the ABI.  The message of the last error on the calling
 *     thread is returned by bscf_last_error().
 *   - One context is not thread-safe; several contexts may coexist.
 */
#ifndef BEADSCF_H
#define BEADSCF_H

#ifdef __cplusplus
extern "C" {
#endif

typedef int bscf_status;
#define BSCF_OK 0
#define BSCF_E_INVALID (-1)     /* bad argument or call order                    */
#define BSCF_E_UNSUPPORTED (-2) /* element/l not in basis, odd electron count, ... */
#define BSCF_E_DEVICE (-3)      /* HIP / rocBLAS / rocSOLVER failure             */
#define BSCF_E_STATE (-4)       /* e.g. forces requested before an SCF           */
#define BSCF_E_NOMEM (-5)       /* device allocation failed                      */

typedef struct bscf_ctx bscf_ctx; /* opaque; owns every device buffer it allocates */

typedef enum { BSCF_FP64 = 0, BSCF_MIXED = 1 } bscf_precision;
typedef enum {
  BSCF_GUESS_CORE = 0,     /* core-Hamiltonian guess                              */
  BSCF_GUESS_PREVIOUS = 1, /* previous SCF orbitals, re-orthonormalised in new S  */
  BSCF_GUESS_LEARNED = 2,  /* density predicted by the in-run trained network     */
  BSCF_GUESS_USER = 3,     /* density set with bscf_set_density                  */
  BSCF_GUESS_EXTRAPOLATED = 4 /* the occupied orbitals of the last two SCFs of each
                          instance extrapolated to second order in the step:
                          C2 aligned to C1 by the orthogonal Procrustes
                          rotation U = polar(C2^T S C1), C = 2 C1 - C2 U,
                          re-orthonormalised in the new S (as the previous-step
                          guess, which it falls back to after one SCF; the core
                          guess before any).  For MD-like sequences of nearby
                          geometries (the reuse of orbitals of Section 2,
                          carried one order further)                          */
} bscf_guess;
typedef enum {
  BSCF_DENSITY_SP2 = 0, /* second-order spectral projection of X^T F X (GEMMs only);
                           a replica without a HOMO-LUMO gap falls back to EIG   */
  BSCF_DENSITY_EIG = 1  /* eigendecomposition of X^T F X with aufbau occupation   */
} bscf_density;

/* Per-instance status bits returned by bscf_run_scf. */
#define BSCF_CONVERGED 0
#define BSCF_MAX_ITER 1
#define BSCF_NAN 2
#define BSCF_FALLBACK_USED 4

typedef struct {
  double e_tol;        /* |E_k - E_{k-1}| threshold (Eh), e.g. 1e-8              */
  double comm_tol;     /* max |X^T(FPS - SPF)X| threshold, e.g. 1e-6 (the paper's
                          density threshold, Section 3.1)                       */
  double schwarz_tol;  /* skip shell quartets with Q_ab Q_cd below this; 1e-12 is
                          the paper's integral cutoff (Section 3.1)              */
  double fp32_split_tol; /* MIXED only: quartets with Q_ab Q_cd above this are
                            evaluated in FP64, the rest in FP32                 */
  int max_iter;        /* SCF iterations per call                               */
  int diis_size;       /* Pulay DIIS subspace (<= 8)                            */
  int precision;       /* bscf_precision                                        */
  int guess;           /* bscf_guess                                            */
  int deterministic;   /* 1: J and K of every Fock build accumulate in exact
                          fixed point (a 128-bit integer with 80 fractional
                          bits per element) instead of FP64 atomics, so they do
                          not depend on the order in which workgroups finish
                          (bitwise equal from run to run at equal densities);
                          0: FP64 atomics (faster; equal to rounding)        */
  int density;         /* bscf_density: how each iteration's density is formed;
                          both give the projector on the lowest N/2 levels of
                          the extrapolated Fock matrix (Section 2, SCF step)   */
  int incremental;     /* 1: iterations after the first build J and K from the
                          density change, skipping quartets whose Schwarz bound
                          times max |dP| is below schwarz_tol (the integral
                          cutoff applied to the change, Section 3.1), with a
                          full build every 12 iterations; 0: every iteration a
                          full build                                            */
  int graph;           /* 1 (with BSCF_DENSITY_SP2): each iteration's steps
                          after its Fock build (commutator error, convergence
                          test, DIIS, SP2 density and its commit) replay a HIP
                          graph that the context captures once per SP2 step
                          count and keeps until the batch changes; the same
                          kernels as with 0, where they are launched one by
                          one; 2: as 1, and each Fock build's J and K
                          accumulation (density change, screening counts,
                          the class kernels on their four streams, the
                          final fold) replays a graph as well, captured once
                          per kind of build until the work lists or the
                          tuning change (a new geometry: new captures)        */
} bscf_scf_opts;

/* Fill opts with defaults: e_tol 1e-8, comm_tol 1e-6, schwarz_tol 1e-12,
 * fp32_split_tol 1e-4, max_iter 100, diis_size 8, FP64, core guess, SP2,
 * incremental builds, graph replay. */
bscf_status bscf_default_opts(bscf_scf_opts* opts);

/* Create a context on HIP device `hip_device`; `hip_stream` may be NULL (the
 * context creates its own) or an existing hipStream_t (not owned). */
bscf_status bscf_create(int hip_device, void* hip_stream, bscf_ctx** out);
bscf_status bscf_destroy(bscf_ctx* ctx);

/* Gaussian basis set of the electronic-structure layer (the paper's runs use
 * 6-31G*, Section 3.1; here with Cartesian d functions).
 * Basis set as JSON text: {"elements": {"H": {"Z": 1, "shells": [{"l": 0,
 * "exponents": [...], "coefficients": [...]}, ...]}, ...}}; s, p, d shells
 * (SP shells given as separate s and p shells).  Copied. */
bscf_status bscf_load_basis(bscf_ctx* ctx, const char* basis_json);

/* The set of n replicas whose BO energies and forces every step needs
 * (Section 2: the PIMD layer generates n nuclear configurations; Section 3.2:
 * the images of a string).
 * Batch composition: n_inst instances; n_atoms[i] atoms each with nuclear
 * charges Z_concat (concatenated over instances) and total charges charge[i]
 * (may be NULL for neutral).  Allocates all per-instance device storage.
 * BSCF_E_UNSUPPORTED for an element missing from the basis or an odd number
 * of electrons, BSCF_E_INVALID for an instance without atoms; arguments are
 * checked before anything changes, so after either the previous instance set
 * and geometry stay usable.  After a device error (BSCF_E_DEVICE,
 * BSCF_E_NOMEM) the context holds no instance set until a call succeeds.
 * A successful call discards the geometry: set it again before computing. */
bscf_status bscf_set_instances(bscf_ctx* ctx, int n_inst, const int* n_atoms,
                               const int* Z_concat, const int* charge);

/* The replicas' configurations of the current step (Section 2), and with them
 * everything that depends on geometry only: the integral screening at the
 * paper's cutoff 1e-12 (Section 3.1) and the one-electron matrices.
 * Nuclear positions [sum n_atoms][3] in bohr, host memory, copied.  Computes
 * the shell-pair data, Schwarz bounds, screened work lists, S, H and the
 * orthogonaliser of every instance on the device. */
bscf_status bscf_set_geometries(bscf_ctx* ctx, const double* xyz_bohr_concat);

/* The direct-SCF Fock build of every replica (the step the paper finds to
 * dominate at high core counts, Section 3.1, Fig. 2b): Roothaan-Hall
 * F = H + J - K/2 (Szabo and Ostlund, Section 3.4) with Schwarz-screened
 * two-electron integrals (cutoff of Section 3.1).
 * One Fock build at given densities: P (all instances concatenated, each
 * n_i x n_i) -> F = H + J - K/2 and E[i] = Tr[P(H+F)]/2 + E_nuc.  With
 * device_ptrs, P and F are device pointers and E may be NULL.  schwarz_tol as
 * in the options (<= 0: no screening); precision a bscf_precision.  The
 * given densities replace the SCF's: bscf_forces then answers BSCF_E_STATE
 * until the next bscf_run_scf (the same holds for bscf_build_jk and
 * bscf_set_density). */
bscf_status bscf_build_fock(bscf_ctx* ctx, const double* P, double* F, double* E,
                            double schwarz_tol, int precision, int device_ptrs);

/* Same build returning J and K separately (for tests). */
bscf_status bscf_build_jk(bscf_ctx* ctx, const double* P, double* J, double* K,
                          double schwarz_tol, int precision, int device_ptrs);

/* The SCF of every replica to the paper's density threshold (Section 3.1),
 * all replicas in one batch; a replica that converges is masked out of later
 * builds, so replicas needing different numbers of SCF cycles do not hold
 * each other up (the imbalance of Section 3.2).
 * Run the SCF of every instance (Pulay DIIS on the orthogonalised commutator;
 * converged when both thresholds hold).  Outputs (host, may be NULL): E[n_inst],
 * n_iter[n_inst], status[n_inst] (bscf status bits).  Non-convergence of an
 * instance is a status bit, not an error. */
bscf_status bscf_run_scf(bscf_ctx* ctx, const bscf_scf_opts* opts, double* E, int* n_iter,
                         int* status);

/* The BO forces of every replica, gathered into one array (Section 2: the
 * forces of the respective replica, summed into the zero-filled per-replica
 * arrays; Fig. 2c).
 * Forces F = -dE/dR [sum n_atoms][3] (Eh/bohr, host) at the densities of the
 * last bscf_run_scf (Pople et al. 1979 gradient with W = P F P / 2; for a
 * B3LYP SCF the Kohn-Sham gradient described at bscf_set_xc).
 * BSCF_E_STATE if no SCF has run at the current geometry or its densities
 * were replaced since. */
bscf_status bscf_forces(bscf_ctx* ctx, double* F);

/* Forces F = -dE/dR [sum n_atoms][3] (Eh/bohr, host) of the same gradient
 * expression as bscf_forces (Pople et al. 1979; the analytic BO force of each
 * replica, Section 2), evaluated at caller densities P and Fock matrices F
 * (all instances concatenated, each n_i x n_i, symmetric; W = P F P / 2)
 * instead of those of an SCF.  Two-electron terms use the screened work lists
 * of the current geometry at Schwarz cutoff schwarz_tol (<= 0: no screening).
 * With device_ptrs, P and F are device pointers; Fout is host memory.  The
 * given densities replace the SCF's, as with bscf_build_fock.  For checking
 * the gradient kernels at densities that do not come from this library. */
bscf_status bscf_forces_at(bscf_ctx* ctx, const double* P, const double* F, double* Fout,
                           double schwarz_tol, int device_ptrs);

/* Ring-polymer (path-integral) molecular dynamics on the device.  The
 * paper's replica layer moves every replica between force calls from its BO
 * force (Section 2; its PIMD of water clusters, Section 3.1, counts time per
 * step as the figure of merit, Fig. 3).  Here the batch's instances are the
 * beads of one ring polymer (copies of one system, at most 64) and the
 * position and momentum update runs on the device in normal-mode
 * coordinates: a step of length dt is O B A B O with the PILE-L Langevin
 * thermostat (Ceriotti, Parrinello, Markland and Manolopoulos 2010) on every
 * normal mode (O), half kicks by the forces (B) and the exact free
 * ring-polymer motion (A).  Convention: physical masses, bead potential V/P,
 * spring frequency w_P = sqrt(P) k_B T / hbar, sampling at T.  The thermostat
 * draws its Gaussian deviates from Philox4x32-10 (Salmon et al. 2011) with
 * the Box-Muller transform, from counters fixed by (seed, step, half-step,
 * mode, atom, xyz), so runs repeat exactly. */
typedef struct {
  double dt;               /* time step, atomic time units (1 fs = 41.341373336)   */
  double temperature;      /* K: the ensemble's, and the spring frequency's        */
  int thermostat;          /* 0: none (NVE); 1: PILE-L                             */
  double tau_centroid;     /* 1/gamma of the centroid mode, atomic time units;
                              <= 0: the centroid is not thermostatted              */
  double friction_scale;   /* lambda in gamma_k = 2 lambda w_k of the internal
                              modes, w_k = 2 w_P sin(k pi / P); 1 = critical       */
  unsigned long long seed; /* key of the thermostat's random stream                */
} bscf_pimd_opts;

/* Defaults: dt 0.25 fs, 300 K, PILE-L, tau_centroid 100 fs, lambda 1, seed 0. */
bscf_status bscf_pimd_default_opts(bscf_pimd_opts* opts);
/* Start a ring polymer at the current geometry (bscf_set_geometries; bead j
 * = instance j) with masses[n_atoms] (electron masses) and momenta p0
 * [P][n_atoms][3] (host; NULL: zero).  BSCF_E_INVALID unless every instance
 * is a copy of instance 0's composition; BSCF_E_UNSUPPORTED above 64 beads.
 * A new batch (bscf_set_instances) ends the ring polymer. */
bscf_status bscf_pimd_init(bscf_ctx* ctx, const bscf_pimd_opts* opts, const double* masses,
                           const double* p0);
/* One step with this context as the force provider: at the first step (or
 * after the positions changed) SCF and forces at the current positions, then
 * O B A, the geometry set from the new positions, the SCF of every bead with
 * opts (E, n_iter, status as bscf_run_scf, host, may be NULL), the forces
 * (-dE/dR [P][n_atoms][3] into `forces`, host, may be NULL), and B O.
 * Learned-guess training, if wanted, is the caller's between steps
 * (bscf_guess_train). */
bscf_status bscf_pimd_step(bscf_ctx* ctx, const bscf_scf_opts* opts, double* E, int* n_iter,
                           int* status, double* forces);
/* The two halves of a step with the caller's forces instead (for other
 * force providers and tests): begin = O B A with forces [P][n_atoms][3]
 * (Eh/bohr, host; -dV/dq of each bead, not divided by P) at the current
 * positions; end = B O with the forces at the new positions.  NULL forces
 * take the context's own, which exist only within bscf_pimd_step
 * (BSCF_E_STATE otherwise).  The context's geometry is not changed. */
bscf_status bscf_pimd_begin(bscf_ctx* ctx, const double* forces);
bscf_status bscf_pimd_end(bscf_ctx* ctx, const double* forces);
/* Positions x and momenta p [P][n_atoms][3] (host, may be NULL) and obs[3]
 * (may be NULL): kinetic energy sum |p|^2/2m, spring energy
 * sum m w_P^2 |q_j - q_{j+1}|^2 / 2 (Eh), and the number of steps taken. */
bscf_status bscf_pimd_state(bscf_ctx* ctx, double* x, double* p, double* obs);

/* Checkpoint and resume of a run between steps.  The paper carries each
 * bead's molecular orbitals from one MD step to the next as the next SCF's
 * starting point (Section 2); a checkpoint writes that carried state, and
 * the ring polymer's, to a file so that a new process continues the run.
 *
 * bscf_checkpoint_save writes (binary, this library's own little-endian
 * format, version 2) the batch's composition, charges and basis sizes, the
 * geometry, the density and the orbitals of the last two SCFs of every
 * instance (the previous-step and extrapolated guesses), the ring polymer if
 * one is running (options, masses, positions, momenta, step count, and the
 * gradient at the current positions when it is held), and the learned
 * guess's network with its Adam moments, its last residual, the previous
 * geometry and its replay buffer of recorded steps.  It needs a geometry
 * (BSCF_E_STATE) and a writable path (BSCF_E_INVALID).
 *
 * bscf_checkpoint_load restores that state into a context whose batch was
 * set with the same composition, charges and basis (bscf_set_instances;
 * BSCF_E_INVALID otherwise, and for a missing, foreign or truncated file,
 * all checked before the context changes): it sets the geometry
 * (bscf_set_geometries), the carried density and orbitals, the ring polymer
 * at its saved step and the network.  The next bscf_pimd_step then takes
 * the same thermostat draws (counters by step) and, with the saved
 * gradient, no extra SCF; the learned guess predicts and trains as it
 * would have.  Not saved: the autotuner's choices (retuned in the new
 * process) and the string method's state; the SCF density has to be
 * recomputed before bscf_forces.
 * With the FP64 path and the previous-step or extrapolated guess the
 * resumed step repeats the uninterrupted one to the rounding of the atomic
 * accumulations (bitwise in the deterministic J/K mode's Fock builds). */
bscf_status bscf_checkpoint_save(bscf_ctx* ctx, const char* path);
bscf_status bscf_checkpoint_load(bscf_ctx* ctx, const char* path);

/* String method on the device.  The paper's second workload moves a
 * reaction path of images between force calls (Section 3.2, Fig. 4: each
 * image's BO energy and force in parallel, images needing different numbers
 * of SCF iterations).  Here the batch's instances are the images (copies of
 * one system, 2..2048) and the path follows the simplified string method
 * (E, Ren and Vanden-Eijnden 2007): every movable image takes the
 * steepest-descent step x <- x + step F, then the images are redistributed
 * to equal arc length along the piecewise-linear path (linear
 * interpolation; the end images keep their positions). */
typedef struct {
  double step;   /* steepest-descent step, bohr^2/Eh (> 0)                 */
  int fix_ends;  /* 1: the first and last image do not move                */
} bscf_string_opts;

/* Defaults: step 0.5 bohr^2/Eh, ends free. */
bscf_status bscf_string_default_opts(bscf_string_opts* opts);
/* Start a string at the current geometry (image i = instance i).
 * BSCF_E_INVALID unless every instance is a copy of instance 0's
 * composition and there are at least two; BSCF_E_UNSUPPORTED above 2048. */
bscf_status bscf_string_init(bscf_ctx* ctx, const bscf_string_opts* opts);
/* One iteration with this context as the force provider: the geometry set
 * from the images (if they moved), the SCF of every image with opts, the
 * forces, then the evolution and redistribution on the device.  E, n_iter,
 * status (as bscf_run_scf) and forces (-dE/dR [n][n_atoms][3]) are those of
 * the images as evaluated, before they move (host, each may be NULL). */
bscf_status bscf_string_step(bscf_ctx* ctx, const bscf_scf_opts* opts, double* E, int* n_iter,
                             int* status, double* forces);
/* The same update with the caller's forces [n][n_atoms][3] (host, Eh/bohr)
 * at the current images, for other force providers and tests. */
bscf_status bscf_string_evolve(bscf_ctx* ctx, const double* forces);
/* Current images [n][n_atoms][3] (bohr) and their normalised arc positions
 * s_i / L [n] (host, each may be NULL). */
bscf_status bscf_string_state(bscf_ctx* ctx, double* x, double* arc);

/* Each replica's converged density, kept on the device between steps (the
 * paper keeps every replica's orbitals in memory for the next step's guess,
 * Section 2).
 * Density of instance `inst` after the last SCF (n_i x n_i), host or device;
 * the last density given to the batch (bscf_set_density, a Fock build) if
 * that came later, and zero before the first of these. */
bscf_status bscf_get_density(bscf_ctx* ctx, int inst, double* P, int device_ptr);
/* Set the density of every instance (concatenated), used by BSCF_GUESS_USER. */
bscf_status bscf_set_density(bscf_ctx* ctx, const double* P, int device_ptrs);
/* One-electron matrices of instance `inst` (host buffers, may be NULL). */
bscf_status bscf_get_one_electron(bscf_ctx* ctx, int inst, double* S, double* H);

/* Full ERI tensor of instance `inst` (n^4 doubles, host), n <= 64; test use
 * (the two-electron integrals behind the Fock build above). */
bscf_status bscf_eri_tensor(bscf_ctx* ctx, int inst, double* out);
/* Schwarz bounds of instance `inst` as an n_shell x n_shell matrix (host). */
bscf_status bscf_schwarz(bscf_ctx* ctx, int inst, double* Q, int nsh);

/* Sizes: basis functions / shells / atoms of instance `inst`. */
bscf_status bscf_instance_info(bscf_ctx* ctx, int inst, int* nbf, int* nshell, int* natom);

/* Counts of the current work lists: screened shell quartets, primitive
 * quartets and the algorithmic FLOPs of one Fock build over all instances. */
bscf_status bscf_work_counts(bscf_ctx* ctx, double* n_quartets, double* n_prim_quartets,
                             double* flops);

/* Deterministic J and K (as bscf_scf_opts.deterministic) for every later
 * Fock build of the context: bscf_build_fock, bscf_build_jk and every SCF
 * (an SCF with opts.deterministic = 1 is deterministic either way). */
bscf_status bscf_set_deterministic(bscf_ctx* ctx, int on);

/* Exchange-correlation model of the Fock builds (the paper's runs use
 * B3LYP, Section 3.1: B3LYP/6-31G*).
 * BSCF_XC_NONE: Hartree-Fock, F = H + J - K/2 (the default).
 * BSCF_XC_B3LYP: closed-shell Kohn-Sham with the B3LYP functional of
 * Stephens, Devlin, Chabalowski and Frisch (1994): F = H + J - 0.1 K + V_xc
 * and E = Tr[P(H + J/2 - 0.05 K)] + E_xc + E_nuc, where E_xc = 0.8 Slater +
 * 0.72 Becke-88 correction + 0.19 VWN (RPA fit) + 0.81 LYP is integrated on
 * a molecular grid of 60 radial x 288 angular points per atom (Becke's radial
 * mapping, R = 1.0 bohr for H and 0.6 bohr otherwise; 12 Gauss-Legendre nodes
 * in cos(theta) x 24 in phi; Becke's fuzzy-cell weights).  Applies to every
 * later bscf_build_fock and bscf_run_scf of the context (bscf_build_jk still
 * returns J and K).  Forces of a B3LYP SCF (bscf_forces, bscf_pimd_step,
 * bscf_string_step; bscf_forces_at while B3LYP is set) are the analytic
 * gradient of that discrete energy: the two-electron term with the exchange
 * scaled by 0.2, W = P F P / 2 from the Kohn-Sham F, and the derivative of
 * E_xc at fixed density with the grid points moving with their atoms,
 * Becke's weight derivatives included.  They need every group of equal basis
 * size to hold instances with the same atoms in the same order (beads,
 * images); otherwise BSCF_E_UNSUPPORTED. */
#define BSCF_XC_NONE 0
#define BSCF_XC_B3LYP 1
bscf_status bscf_set_xc(bscf_ctx* ctx, int functional);

/* The B3LYP exchange-correlation matrix and energy (Section 3.1's level of
 * theory; the grid and functional of bscf_set_xc) at densities P (all
 * instances concatenated, each n_i x n_i, symmetric): Vxc[i] (n_i x n_i) and
 * Exc[i] per instance.  With device_ptrs all three are device pointers.  The
 * given densities replace the SCF's, as with bscf_build_fock. */
bscf_status bscf_xc_matrix(bscf_ctx* ctx, const double* P, double* Vxc, double* Exc,
                           int device_ptrs);

/* Number of grid points of instance `inst` (atoms x 17280). */
bscf_status bscf_xc_grid_size(bscf_ctx* ctx, int inst, long long* npts);

/* The closed-shell B3LYP energy density e(rho, sigma) (Eh/bohr^3) and its
 * derivatives vrho = de/drho, vsigma = de/dsigma at n points on the device
 * (rho the total density, sigma = |grad rho|^2; host arrays).  rho must be
 * positive.  Test use. */
bscf_status bscf_xc_functional(bscf_ctx* ctx, int n, const double* rho, const double* sigma,
                               double* e, double* vrho, double* vsigma);

/* Kernel profiling: with on != 0 every Fock-build class kernel is bracketed by
 * HIP events on the context's stream; per-class times appear in the stats. */
bscf_status bscf_set_profiling(bscf_ctx* ctx, int on);
/* Zero the accumulated counters and timers reported by bscf_get_stats. */
bscf_status bscf_reset_stats(bscf_ctx* ctx);

/* Timings behind the paper's figure of merit, time per step (Section 3.1,
 * Fig. 3), split by phase and by integral class.
 * Statistics as a JSON object: per quartet class the screened quartet and
 * primitive-quartet counts of the current work lists, the counts and
 * algorithmic FLOPs evaluated since the last reset (active instances only) and
 * the measured kernel time; totals of Fock builds, SCF iterations and phase
 * timers (ms). */
bscf_status bscf_get_stats(bscf_ctx* ctx, char* buf, int len);

/* Evaluate the device Boys function: out[i*(m_max+1)+m] = F_m(T[i]) for n
 * values of T (host arrays), in FP64 (precision 0) or FP32 (1).  Test use. */
bscf_status bscf_boys(bscf_ctx* ctx, int m_max, int n, const double* T, double* out,
                      int precision);
/* Host-side Boys table entry F_m(0.1 k) used to build the device table. */
double bscf_boys_table_entry(int m, int k);

/* Learned SCF guess.  The paper reuses each replica's previous-step orbitals
 * as the next step's starting point (Section 2); the learned guess corrects
 * that previous-step density with a network over atom pairs (inputs: the
 * pair's element types, geometry and displacement, its block of the
 * previous-step guess and of the previous step's residual; output: the
 * residual block, converged minus previous-step density), trained in-run.
 * Every converged SCF that started from the previous-step, extrapolated or
 * learned guess records its residual rows; run_scf with BSCF_GUESS_LEARNED applies the
 * network once it has been trained, and otherwise (no model, no previous
 * step, or a non-finite or oversized prediction) keeps the previous-step
 * guess and sets BSCF_FALLBACK_USED.  The converged result does not depend on
 * the guess beyond the SCF tolerance.
 *
 * Network: din -> 256 -> 256 -> dout, ReLU, FP32, plus a residual connection
 * (the last dout inputs are added to the output; dout <= din); loss = masked
 * mean squared error; Adam (beta 0.9 / 0.999, eps 1e-8).  Flat parameter
 * order: W1 (din x 256, row-major), b1, W2 (256 x 256), b2, W3 (256 x dout),
 * b3. */

/* n_adam_steps full-batch Adam steps (learning rate 1e-3) on the last four
 * recorded steps; *loss = loss before the last step (negative: no data). */
bscf_status bscf_guess_train(bscf_ctx* ctx, int n_adam_steps, float* loss);
/* Model, residual scale and Adam state to / from a binary file. */
bscf_status bscf_guess_save(bscf_ctx* ctx, const char* path);
bscf_status bscf_guess_load(bscf_ctx* ctx, const char* path);
/* Fix the network to din inputs and dout outputs with seeded initial weights
 * (in-run use sizes it from the batch by itself). */
bscf_status bscf_guess_configure(bscf_ctx* ctx, int din, int dout, unsigned seed);
/* Current input and output widths and parameter count (0 when unconfigured). */
bscf_status bscf_guess_param_count(bscf_ctx* ctx, int* din, int* dout, long* n);
/* Copy the flat parameter vector in / out (host, n floats); setting resets
 * the Adam moments.  BSCF_E_INVALID if n differs from the parameter count. */
bscf_status bscf_guess_set_params(bscf_ctx* ctx, const float* params, long n);
bscf_status bscf_guess_get_params(bscf_ctx* ctx, float* params, long n);
/* Evaluate the network on rows x din host inputs X into Y (rows x dout, may
 * be NULL); with targets T and mask (rows x dout, both or neither) also the
 * loss and the flat gradient (grad: parameter count floats, may be NULL). */
bscf_status bscf_guess_eval(bscf_ctx* ctx, int rows, const float* X, const float* T,
                            const float* mask, float* Y, float* grad, float* loss);
/* steps full-batch Adam steps with learning rate lr on the given rows, from
 * the current moments; *loss = loss before the last step. */
bscf_status bscf_guess_fit(bscf_ctx* ctx, int rows, const float* X, const float* T,
                           const float* mask, int steps, float lr, float* loss);

/* Allocation-free evaluation of the guess network, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The same result as bscf_guess_eval
 * without targets: Y = net(X) for `rows` input rows.  X (rows x din) and Y
 * (rows x dout) are FP32 row-major HIP device pointers on the context's
 * device; the work is enqueued on the context's stream and the call returns
 * without synchronising.  It allocates nothing: the hidden activations go to
 * one fixed array per GPU of 2 x BSCF_NOALLOC_MAX_ROWS x 256 floats (16 MiB),
 * set up by bscf_create and held until the process ends.  rows must be
 * 1..BSCF_NOALLOC_MAX_ROWS (BSCF_E_INVALID otherwise); BSCF_E_STATE without a
 * configured network.  Every call on one GPU uses that GPU's array, so calls
 * that overlap on one GPU (other contexts or streams) race; calls ordered on
 * one stream do not. */
#define BSCF_NOALLOC_MAX_ROWS 8192
bscf_status bscf_guess_eval_noalloc(bscf_ctx* ctx, int rows, const float* X, float* Y);

/* Message of the last failed call on this thread ("" if none). */
const char* bscf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BEADSCF_H */
