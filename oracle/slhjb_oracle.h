/*
 * FP64 CPU oracle for the semi-Lagrangian Markov-chain scheme of Cacace & Falcone,
 * "A dynamic domain decomposition for a class of second order semi-linear equations".
 *
 * TEST INFRASTRUCTURE ONLY. This is the plain, slow reference that the GPU library is
 * checked against. Only the test-suite, the smoke check and the benchmark's CPU-baseline
 * leg may load it. It shares no code, header, table or helper with the GPU library.
 *
 * All arithmetic is IEEE double except where the method turns floating point into an
 * integer (the Q.8 foot displacement of the labeler), which is done in float exactly as
 * documented at or_displacement().
 */
#ifndef SLHJB_ORACLE_H
#define SLHJB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_FREE = 0, OR_TARGET = 1, OR_OBSTACLE = 2 };
enum { OR_DIFF_NONE = 0, OR_DIFF_ISO = 1, OR_DIFF_RANK1 = 2 };
enum { OR_SL2 = 0, OR_SL3 = 1 };

/* A discrete problem on the n x n node grid of [x_lo,x_hi]^2, node (i,j) at
 * (x_lo+i*dx, x_lo+j*dx), stored row-major at j*n+i. Dynamics f(x,a)=c(x)(d(x)+a), with the
 * drift d = 0 when drift is NULL (Section 5: A is a pure drift, B has none, C both). */
typedef struct {
    int32_t n;
    double x_lo, x_hi;
    double h;              /* time step of the scheme */
    double lambda;         /* discount rate (>= 0; 0 = the undiscounted scheme of Section 3) */
    double eps;            /* diffusion coefficient (when eps_field is NULL) */
    int32_t diffusion;     /* OR_DIFF_* */
    int32_t scheme;        /* OR_SL2 / OR_SL3 */
    int32_t n_controls;
    const double* controls;        /* [2*n_controls], a_m = (controls[2m], controls[2m+1]) */
    const double* speed;           /* [n*n] c(x_i) > 0 */
    double running_cost;           /* l (constant) */
    const uint8_t* node_class;     /* [n*n] OR_FREE / OR_TARGET / OR_OBSTACLE */
    double target_value;           /* g on TARGET nodes */
    double v_out;                  /* value at feet outside the closed box; held by OBSTACLE nodes */
    const double* drift;           /* [2*n*n] (d_1, d_2) per node, or NULL */
    /* Section 5.2-5.3: costs and diffusion that depend on the state and the control. The
     * running cost is l(x,a) = l_x(x) + l_a(a) (the paper's l_1, l_2, l_3 all have this form);
     * the diffusion coefficient may vary over the nodes (eps(x), degenerate where it is 0). */
    const double* running_cost_field;  /* [n*n] l_x per node, or NULL = running_cost */
    const double* control_cost;        /* [n_controls] l_a per control, or NULL = 0 */
    const double* eps_field;           /* [n*n] eps(x) per node, or NULL = eps */
} or_problem;

double or_beta(const or_problem* p);
double or_rho(const or_problem* p);
double or_rho_at(const or_problem* p, int32_t node, int32_t m);
int32_t or_feet(const or_problem* p, int32_t i, int32_t j, int32_t m, double* y /* [4][2] */);
int32_t or_interp_weights(const or_problem* p, double y1, double y2, int32_t* idx /*[4]*/, double* w /*[4]*/);
double or_interp(const or_problem* p, const double* v, double y1, double y2);
double or_one_step_mean(const or_problem* p, const double* v, int32_t node, int32_t m);
double or_candidate(const or_problem* p, const double* v, int32_t node, int32_t m);
double or_bellman(const or_problem* p, const double* v, int32_t node, int32_t* argmin);
double or_jacobi_sweep(const or_problem* p, const double* v_in, double* v_out, int32_t n_threads);
int64_t or_solve(const or_problem* p, double* v, double tol, int64_t max_sweeps, int32_t gauss_seidel,
                 const int32_t* order, int32_t n_threads, double* residual_out,
                 double* history, int64_t history_len);
int32_t or_transitions(const or_problem* p, int32_t node, int32_t m, int32_t* idx /*[16]*/,
                       double* w /*[16]*/, double* w_out);
void or_policy_chain(const or_problem* p, const int32_t* policy, int32_t* idx /*[N][16]*/, double* w /*[N][16]*/,
                     double* w_out /*[N]*/, int32_t n_threads);
void or_rho_policy(const or_problem* p, const int32_t* policy, double* out /*[N]*/);
int64_t or_policy_improve(const or_problem* p, const double* v, int32_t* policy, int32_t n_threads);
void or_synthesize(const or_problem* p, const double* v_hat, int32_t* ctrl_out, double* gap_out);
void or_upsample_bilinear(int32_t n_c, const double* v_c, int32_t n_f, double* v_f);
void or_upsample_bicubic(int32_t n_c, const double* v_c, int32_t n_f, double* v_f);
void or_displacement(int32_t n, float x_lo, float x_hi, float h, const float* speed,
                     const float* controls, const int32_t* ctrl, int32_t* disp_q8);
int64_t or_label(int32_t n, const uint8_t* node_class, const int32_t* disp_q8, const int16_t* source_patch,
                 int32_t n_patches, int32_t order_mode, uint16_t* phi, int16_t* label);
double or_sweep_independent(const or_problem* p, const int16_t* label, const double* v_in, double* v_out,
                            int32_t n_threads);

#ifdef __cplusplus
}
#endif
#endif
