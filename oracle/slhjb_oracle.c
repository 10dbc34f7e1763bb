/*
 * FP64 CPU oracle for the semi-Lagrangian Markov-chain scheme (Cacace & Falcone,
 * arXiv 1502.01629).
 *
 * TEST INFRASTRUCTURE ONLY: the plain, slow, obviously correct reference that the GPU
 * library is checked against. It is loaded by the tests, the smoke check and the CPU
 * baseline of the benchmark, and by nothing on the product path. It shares no code with
 * the GPU library. Every function follows the definition it cites literally: no blocking,
 * no fusion, no reordering beyond what the definition states.
 *
 * Discrete problem (the scheme of Section 3, eq. SLscheme2, in discounted Kruzkov form):
 *   feet     y = x_i + h c(x_i) a + s sqrt(h) sigma_k(x_i,a),  s = +-1, k = 1..d
 *   SL2      v_i = min_a [ beta * (1/2d) sum_{k,s} I[v](y) + rho ]
 *   SL3      v_i = min_a (beta Lambda1(a) + rho) / (1 - beta Lambda0(a))     (eq. SLscheme3)
 * with beta = fl32(exp(-lambda h)), rho = (1-beta) l / lambda for lambda > 0, and for
 * lambda = 0 beta = 1, rho = h l: the undiscounted scheme exactly as printed in Section 3.
 * The running cost l(x,a) = l_x(x) + l_a(a) and the diffusion coefficient eps(x) may vary
 * (Sections 5.2-5.3).
 */
#include "slhjb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static double or_dx(const or_problem* p) { return (p->x_hi - p->x_lo) / (double)(p->n - 1); }

/* The discount factor of one time step, exp(-lambda h). The GPU computes in float, so the
 * discrete problem both sides solve carries the float rounding of this number. */
double or_beta(const or_problem* p) { return (double)(float)exp(-p->lambda * p->h); }

/* Running cost collected over one step: (1-beta) l / lambda in the discounted form, h l in the
 * undiscounted one (lambda = 0, eq. SLscheme2 as printed). */
static double or_step_cost(const or_problem* p, double l) {
    if (p->lambda == 0.0) return p->h * l;
    return (1.0 - or_beta(p)) * l / p->lambda;
}

/* For a constant running cost (no per-node or per-control part). */
double or_rho(const or_problem* p) { return or_step_cost(p, p->running_cost); }

/* At FREE node `node` under control m: l(x,a) = l_x(x_node) + l_a(a_m). */
double or_rho_at(const or_problem* p, int32_t node, int32_t m) {
    double l = p->running_cost_field ? p->running_cost_field[node] : p->running_cost;
    if (p->control_cost) l += p->control_cost[m];
    return or_step_cost(p, l);
}

/* Feet of node (i,j) under control m (eq. SLscheme2, first line). Dynamics
 * f = c(x) (d(x) + a): the drift d of the advection and Zermelo examples (Section 5), 0 if absent.
 * NONE : sigma = 0, the 2d feet coincide, one foot.
 * ISO  : sigma = sqrt(2 eps) I, feet x + h f +- sqrt(2 eps h) e_k, k = 1,2 (Section 4.1).
 * RANK1: sigma(x,a) = sqrt(2 eps) a, one noise direction, feet x + h f +- sqrt(2 eps h) a
 *        (the control-driven diffusion sigma_3 of Section 5.3).
 * Returns the number of feet K and writes them to y[2*k], y[2*k+1]. */
int32_t or_feet(const or_problem* p, int32_t i, int32_t j, int32_t m, double* y) {
    const double dx = or_dx(p);
    const double x1 = p->x_lo + i * dx;
    const double x2 = p->x_lo + j * dx;
    const double c = p->speed[(int64_t)j * p->n + i];
    const double a1 = p->controls[2 * m];
    const double a2 = p->controls[2 * m + 1];
    const double d1 = p->drift ? p->drift[2 * ((int64_t)j * p->n + i)] : 0.0;
    const double d2 = p->drift ? p->drift[2 * ((int64_t)j * p->n + i) + 1] : 0.0;
    const double b1 = x1 + p->h * c * (d1 + a1);
    const double b2 = x2 + p->h * c * (d2 + a2);
    const double eps = p->eps_field ? p->eps_field[(int64_t)j * p->n + i] : p->eps;
    const double d = sqrt(2.0 * eps * p->h);
    switch (p->diffusion) {
    case OR_DIFF_ISO:
        y[0] = b1 + d; y[1] = b2;
        y[2] = b1 - d; y[3] = b2;
        y[4] = b1;     y[5] = b2 + d;
        y[6] = b1;     y[7] = b2 - d;
        return 4;
    case OR_DIFF_RANK1:
        y[0] = b1 + d * a1; y[1] = b2 + d * a2;
        y[2] = b1 - d * a1; y[3] = b2 - d * a2;
        return 2;
    default:
        y[0] = b1; y[1] = b2;
        return 1;
    }
}

/* Bilinear reconstruction at y (Section 3, Fig. bilinear): the four nodes of the cell that
 * holds y and their weights (1-s)(1-t), s(1-t), (1-s)t, st. The cell index is clamped to
 * n-2 so that points on the upper edge use the last cell. Returns 0 if y lies outside the
 * closed box (no weights), 1 otherwise. */
int32_t or_interp_weights(const or_problem* p, double y1, double y2, int32_t* idx, double* w) {
    const int32_t n = p->n;
    if (y1 < p->x_lo || y1 > p->x_hi || y2 < p->x_lo || y2 > p->x_hi) return 0;
    const double dx = or_dx(p);
    const double q1 = (y1 - p->x_lo) / dx;
    const double q2 = (y2 - p->x_lo) / dx;
    int32_t c1 = (int32_t)floor(q1);
    int32_t c2 = (int32_t)floor(q2);
    if (c1 > n - 2) c1 = n - 2;
    if (c2 > n - 2) c2 = n - 2;
    if (c1 < 0) c1 = 0;
    if (c2 < 0) c2 = 0;
    const double s = q1 - c1;
    const double t = q2 - c2;
    idx[0] = c2 * n + c1;
    idx[1] = c2 * n + c1 + 1;
    idx[2] = (c2 + 1) * n + c1;
    idx[3] = (c2 + 1) * n + c1 + 1;
    w[0] = (1.0 - s) * (1.0 - t);
    w[1] = s * (1.0 - t);
    w[2] = (1.0 - s) * t;
    w[3] = s * t;
    return 1;
}

/* I[v](y), with the value v_out outside the closed box. */
double or_interp(const or_problem* p, const double* v, double y1, double y2) {
    int32_t idx[4];
    double w[4];
    if (!or_interp_weights(p, y1, y2, idx, w)) return p->v_out;
    return w[0] * v[idx[0]] + w[1] * v[idx[1]] + w[2] * v[idx[2]] + w[3] * v[idx[3]];
}

/* (1/2d) sum_{k,s} I[v](y): the expected value after one step of the Markov chain. */
double or_one_step_mean(const or_problem* p, const double* v, int32_t node, int32_t m) {
    double y[8];
    const int32_t K = or_feet(p, node % p->n, node / p->n, m, y);
    double sum = 0.0;
    for (int32_t k = 0; k < K; ++k) sum += or_interp(p, v, y[2 * k], y[2 * k + 1]);
    return sum / K;
}

/* The candidate value of control m at a FREE node: the bracket of eq. SLscheme2 (SL2) or the
 * quotient of eq. SLscheme3 (SL3). For SL3, Lambda0 collects the node's own interpolation
 * weights over the feet and Lambda1 everything else (eq. SLimplicit); a node that is not a
 * corner of a foot's cell has weight 0 there, and a foot outside the box contributes v_out
 * with weight 1 to Lambda1. */
double or_candidate(const or_problem* p, const double* v, int32_t node, int32_t m) {
    const double beta = or_beta(p);
    const double rho = or_rho_at(p, node, m);
    double y[8];
    const int32_t K = or_feet(p, node % p->n, node / p->n, m, y);
    double mean = 0.0, lam0 = 0.0, lam1 = 0.0;
    for (int32_t k = 0; k < K; ++k) {
        int32_t idx[4];
        double w[4];
        if (!or_interp_weights(p, y[2 * k], y[2 * k + 1], idx, w)) {
            mean += p->v_out;
            lam1 += p->v_out;
            continue;
        }
        for (int32_t c = 0; c < 4; ++c) {
            mean += w[c] * v[idx[c]];
            if (idx[c] == node) lam0 += w[c];
            else lam1 += w[c] * v[idx[c]];
        }
    }
    mean /= K;
    lam0 /= K;
    lam1 /= K;
    if (p->scheme == OR_SL3) return (beta * lam1 + rho) / (1.0 - beta * lam0);
    return beta * mean + rho;
}

/* Min over the discrete control set by direct comparison (Section 3); the first minimum wins. */
double or_bellman(const or_problem* p, const double* v, int32_t node, int32_t* argmin) {
    double best = INFINITY;
    int32_t bm = -1;
    for (int32_t m = 0; m < p->n_controls; ++m) {
        const double q = or_candidate(p, v, node, m);
        if (q < best) { best = q; bm = m; }
    }
    if (argmin) *argmin = bm;
    return best;
}

static double or_fixed_value(const or_problem* p, uint8_t cls) {
    return cls == OR_TARGET ? p->target_value : p->v_out;
}

/* One Jacobi sweep: every FREE node from v_in, TARGET and OBSTACLE nodes keep their data.
 * Returns the sup-norm change over FREE nodes. */
double or_jacobi_sweep(const or_problem* p, const double* v_in, double* v_out, int32_t n_threads) {
    const int64_t N = (int64_t)p->n * p->n;
    double resid = 0.0;
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for reduction(max : resid) num_threads(n_threads) schedule(dynamic, 64)
    for (int64_t node = 0; node < N; ++node) {
        const uint8_t cls = p->node_class[node];
        if (cls != OR_FREE) {
            v_out[node] = or_fixed_value(p, cls);
            continue;
        }
        const double q = or_bellman(p, v_in, (int32_t)node, NULL);
        v_out[node] = q;
        const double d = fabs(q - v_in[node]);
        if (d > resid) resid = d;
    }
    return resid;
}

/* Value iteration until the sup-norm change is <= tol (the convergence test of the patchy
 * algorithm, Section 4.3) or max_sweeps. Jacobi uses two buffers; Gauss-Seidel updates in
 * place in the given order (row-major if order is NULL). Returns the number of sweeps. */
int64_t or_solve(const or_problem* p, double* v, double tol, int64_t max_sweeps, int32_t gauss_seidel,
                 const int32_t* order, int32_t n_threads, double* residual_out,
                 double* history, int64_t history_len) {
    const int64_t N = (int64_t)p->n * p->n;
    for (int64_t node = 0; node < N; ++node)
        if (p->node_class[node] != OR_FREE) v[node] = or_fixed_value(p, p->node_class[node]);
    double* tmp = NULL;
    if (!gauss_seidel) {
        tmp = (double*)malloc(sizeof(double) * N);
        if (!tmp) return -1;
    }
    double r = INFINITY;
    int64_t s = 0;
    while (s < max_sweeps) {
        if (gauss_seidel) {
            r = 0.0;
            for (int64_t q = 0; q < N; ++q) {
                const int32_t node = order ? order[q] : (int32_t)q;
                if (p->node_class[node] != OR_FREE) continue;
                const double val = or_bellman(p, v, node, NULL);
                const double d = fabs(val - v[node]);
                if (d > r) r = d;
                v[node] = val;
            }
        } else {
            r = or_jacobi_sweep(p, v, tmp, n_threads);
            memcpy(v, tmp, sizeof(double) * N);
        }
        if (history && s < history_len) history[s] = r;
        ++s;
        if (r <= tol) break;
    }
    free(tmp);
    if (residual_out) *residual_out = r;
    return s;
}

/* The Markov chain of control m at a node (Section 3): for every foot, the four cell nodes
 * with weight w/K; the weight of feet outside the box goes to *w_out. Entries are listed per
 * foot and corner, without merging repeated nodes. Returns the number of entries. */
int32_t or_transitions(const or_problem* p, int32_t node, int32_t m, int32_t* idx, double* w, double* w_out) {
    double y[8];
    const int32_t K = or_feet(p, node % p->n, node / p->n, m, y);
    int32_t cnt = 0;
    *w_out = 0.0;
    for (int32_t k = 0; k < K; ++k) {
        int32_t ci[4];
        double cw[4];
        if (!or_interp_weights(p, y[2 * k], y[2 * k + 1], ci, cw)) {
            *w_out += 1.0 / K;
            continue;
        }
        for (int32_t c = 0; c < 4; ++c) {
            idx[cnt] = ci[c];
            w[cnt] = cw[c] / K;
            ++cnt;
        }
    }
    return cnt;
}

/* Howard's policy iteration, the pieces that touch every node (Section 3 scheme as a Markov
 * decision problem): the chain of a policy at every node, and the greedy improvement step. */

/* For every node: up to 16 (index, weight) pairs of the chain of control policy[node] (padded
 * with index -1), and the weight of feet outside the box. Nodes that are not FREE get no entries. */
void or_policy_chain(const or_problem* p, const int32_t* policy, int32_t* idx, double* w, double* w_out,
                     int32_t n_threads) {
    const int64_t N = (int64_t)p->n * p->n;
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for num_threads(n_threads) schedule(dynamic, 256)
    for (int64_t node = 0; node < N; ++node) {
        int32_t* ri = idx + 16 * node;
        double* rw = w + 16 * node;
        for (int32_t k = 0; k < 16; ++k) { ri[k] = -1; rw[k] = 0.0; }
        w_out[node] = 0.0;
        if (p->node_class[node] != OR_FREE) continue;
        or_transitions(p, (int32_t)node, policy[node], ri, rw, &w_out[node]);
    }
}

/* The step cost of every node under its control policy[node] (0 on nodes that are not FREE). */
void or_rho_policy(const or_problem* p, const int32_t* policy, double* out) {
    const int64_t N = (int64_t)p->n * p->n;
    for (int64_t node = 0; node < N; ++node)
        out[node] = p->node_class[node] == OR_FREE ? or_rho_at(p, (int32_t)node, policy[node]) : 0.0;
}

/* Greedy improvement at v: every FREE node takes a control of smallest eq. SLscheme2 candidate,
 * keeping its current control unless another one is smaller by more than a relative 1e-14.
 * Returns the number of nodes whose control changed. */
int64_t or_policy_improve(const or_problem* p, const double* v, int32_t* policy, int32_t n_threads) {
    const int64_t N = (int64_t)p->n * p->n;
    or_problem q = *p;
    q.scheme = OR_SL2;
    int64_t changed = 0;
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for reduction(+ : changed) num_threads(n_threads) schedule(dynamic, 64)
    for (int64_t node = 0; node < N; ++node) {
        if (p->node_class[node] != OR_FREE) continue;
        int32_t bm = 0;
        const double best = or_bellman(&q, v, (int32_t)node, &bm);
        const double cur = or_candidate(&q, v, (int32_t)node, policy[node]);
        const double scale = fabs(cur) > 1.0 ? fabs(cur) : 1.0;
        if (best < cur - 1e-14 * scale) {
            policy[node] = bm;
            ++changed;
        }
    }
    return changed;
}

/* Discrete synthesis of the feedback control (Section 4.3, eq. discrete-synthesis) with
 * sigma = 0 and a constant running cost: argmin over controls of I[v_hat](x_i + h c a).
 * The first minimum wins. gap_out (nullable) receives second-best minus best, so callers can
 * tell genuine ties. Nodes that are not FREE get -1. */
void or_synthesize(const or_problem* p, const double* v_hat, int32_t* ctrl_out, double* gap_out) {
    const int64_t N = (int64_t)p->n * p->n;
    const double dx = or_dx(p);
    for (int64_t node = 0; node < N; ++node) {
        if (p->node_class[node] != OR_FREE) {
            ctrl_out[node] = -1;
            if (gap_out) gap_out[node] = INFINITY;
            continue;
        }
        const int32_t i = (int32_t)(node % p->n), j = (int32_t)(node / p->n);
        const double x1 = p->x_lo + i * dx, x2 = p->x_lo + j * dx;
        const double c = p->speed[node];
        double best = INFINITY, second = INFINITY;
        int32_t bm = -1;
        for (int32_t m = 0; m < p->n_controls; ++m) {
            const double d1 = p->drift ? p->drift[2 * node] : 0.0;
            const double d2 = p->drift ? p->drift[2 * node + 1] : 0.0;
            const double q = or_interp(p, v_hat, x1 + p->h * c * (d1 + p->controls[2 * m]),
                                       x2 + p->h * c * (d2 + p->controls[2 * m + 1]));
            if (q < best) { second = best; best = q; bm = m; }
            else if (q < second) second = q;
        }
        ctrl_out[node] = bm;
        if (gap_out) gap_out[node] = second - best;
    }
}

/* u_hat on the fine grid by bilinear interpolation of the coarse solution (Section 4.3,
 * "by interpolation"). Both grids cover the same box with n-1 cells per side. */
void or_upsample_bilinear(int32_t n_c, const double* v_c, int32_t n_f, double* v_f) {
    const double ratio = (double)(n_c - 1) / (double)(n_f - 1);
    for (int32_t j = 0; j < n_f; ++j) {
        for (int32_t i = 0; i < n_f; ++i) {
            const double q1 = i * ratio, q2 = j * ratio;
            int32_t c1 = (int32_t)floor(q1), c2 = (int32_t)floor(q2);
            if (c1 > n_c - 2) c1 = n_c - 2;
            if (c2 > n_c - 2) c2 = n_c - 2;
            const double s = q1 - c1, t = q2 - c2;
            v_f[(int64_t)j * n_f + i] = (1 - s) * (1 - t) * v_c[c2 * n_c + c1] + s * (1 - t) * v_c[c2 * n_c + c1 + 1] +
                                        (1 - s) * t * v_c[(c2 + 1) * n_c + c1] + s * t * v_c[(c2 + 1) * n_c + c1 + 1];
        }
    }
}

/* Keys' cubic convolution kernel with a = -1/2 (R. G. Keys, "Cubic convolution interpolation
 * for digital image processing", IEEE Trans. ASSP 29 (1981), eq. 15):
 *   W(x) = (a+2)|x|^3 - (a+3)|x|^2 + 1          for |x| <= 1,
 *          a|x|^3 - 5a|x|^2 + 8a|x| - 4a         for 1 < |x| < 2,  0 otherwise. */
static double or_keys(double x) {
    const double a = -0.5;
    const double t = fabs(x);
    if (t <= 1.0) return (a + 2.0) * t * t * t - (a + 3.0) * t * t + 1.0;
    if (t < 2.0) return a * t * t * t - 5.0 * a * t * t + 8.0 * a * t - 4.0 * a;
    return 0.0;
}

/* Bicubic (Keys) interpolation of a coarse grid solution onto a fine grid of the same box, the
 * feature of the learned warm start: fine node i at coarse coordinate q = i (n_c-1)/(n_f-1),
 * base cell c = floor(q) (c = n_c-2 on the upper edge), fraction t = q - c, and the 4 x 4 coarse
 * nodes c-1..c+2 per axis weighted by W(t - m), m = -1..2; indices outside the grid are clamped
 * to the nearest edge node (edge replication). */
void or_upsample_bicubic(int32_t n_c, const double* v_c, int32_t n_f, double* v_f) {
    const double ratio = (double)(n_c - 1) / (double)(n_f - 1);
    for (int32_t j = 0; j < n_f; ++j) {
        for (int32_t i = 0; i < n_f; ++i) {
            const double q1 = i * ratio, q2 = j * ratio;
            int32_t c1 = (int32_t)floor(q1), c2 = (int32_t)floor(q2);
            if (c1 > n_c - 2) c1 = n_c - 2;
            if (c2 > n_c - 2) c2 = n_c - 2;
            const double s = q1 - c1, t = q2 - c2;
            double sum = 0.0;
            for (int32_t my = -1; my <= 2; ++my) {
                int32_t y = c2 + my;
                if (y < 0) y = 0;
                if (y > n_c - 1) y = n_c - 1;
                for (int32_t mx = -1; mx <= 2; ++mx) {
                    int32_t x = c1 + mx;
                    if (x < 0) x = 0;
                    if (x > n_c - 1) x = n_c - 1;
                    sum += or_keys(s - mx) * or_keys(t - my) * v_c[(int64_t)y * n_c + x];
                }
            }
            v_f[(int64_t)j * n_f + i] = sum;
        }
    }
}

/* The foot of the synthesized dynamics x_i + h c(x_i) a*(x_i) (eq. discrete-advection) as a
 * Q.8 fixed-point displacement in cell units. This is where floating point decides integers,
 * so it is computed in float exactly as the GPU does:
 *   dx32 = fl((x_hi - x_lo) / (n-1)),  r = fl(h / dx32),  k = fl(r * c_i),
 *   D = round_half_even(256 * fl(k * a)) per axis.
 * Nodes with ctrl < 0 get D = 0. */
void or_displacement(int32_t n, float x_lo, float x_hi, float h, const float* speed,
                     const float* controls, const int32_t* ctrl, int32_t* disp_q8) {
    volatile float span = x_hi - x_lo;
    volatile float dx32 = span / (float)(n - 1);
    volatile float r = h / dx32;
    const int64_t N = (int64_t)n * n;
    for (int64_t node = 0; node < N; ++node) {
        const int32_t m = ctrl[node];
        if (m < 0) {
            disp_q8[2 * node] = 0;
            disp_q8[2 * node + 1] = 0;
            continue;
        }
        volatile float k = r * speed[node];
        volatile float px = k * controls[2 * m];
        volatile float py = k * controls[2 * m + 1];
        volatile float sx = 256.0f * px;
        volatile float sy = 256.0f * py;
        disp_q8[2 * node] = (int32_t)rintf(sx);
        disp_q8[2 * node + 1] = (int32_t)rintf(sy);
    }
}

/* Integer form of the patch construction (Section 4.3, eq. discrete-advection and the
 * thresholding that follows). phi_p holds values in [0, 2^15]: 2^15 on the source nodes of
 * patch p, 0 on other sources, obstacles and outside the box. A FREE node takes the
 * bilinear value of phi_p at its synthesized foot, with weights (256-f or f) per axis that
 * sum to 2^16, rounded half up:  phi'(x) = (sum_c W_c phi(c) + 2^15) >> 16.
 * The map is monotone and the start is below its image, so any fair update order climbs to
 * the same least fixed point; iteration stops when nothing changes (order_mode 0 = Jacobi,
 * 1 = in place row-major, 2 = in place reversed). label = argmax_p phi_p (lowest p on ties),
 * -1 where every phi_p is 0. Returns the number of passes, including the last one that
 * changed nothing. */
int64_t or_label(int32_t n, const uint8_t* node_class, const int32_t* disp_q8, const int16_t* source_patch,
                 int32_t n_patches, int32_t order_mode, uint16_t* phi, int16_t* label) {
    const int64_t N = (int64_t)n * n;
    const int32_t P = n_patches;
    const uint32_t ONE = 1u << 15;
    memset(phi, 0, sizeof(uint16_t) * N * P);
    for (int64_t node = 0; node < N; ++node)
        if (node_class[node] == OR_TARGET && source_patch[node] >= 0) phi[node * P + source_patch[node]] = (uint16_t)ONE;
    uint16_t* prev = NULL;
    if (order_mode == 0) {
        prev = (uint16_t*)malloc(sizeof(uint16_t) * N * P);
        if (!prev) return -1;
    }
    int64_t passes = 0;
    for (;;) {
        int changed = 0;
        if (prev) memcpy(prev, phi, sizeof(uint16_t) * N * P);
        const uint16_t* src = prev ? prev : phi;
        for (int64_t q = 0; q < N; ++q) {
            const int64_t node = order_mode == 2 ? N - 1 - q : q;
            if (node_class[node] != OR_FREE) continue;
            const int32_t i = (int32_t)(node % n), j = (int32_t)(node / n);
            const int32_t Dx = disp_q8[2 * node], Dy = disp_q8[2 * node + 1];
            const int32_t ci = i + (Dx >> 8), cj = j + (Dy >> 8);
            const uint32_t fx = (uint32_t)(Dx & 255), fy = (uint32_t)(Dy & 255);
            const uint32_t W[4] = {(256 - fx) * (256 - fy), fx * (256 - fy), (256 - fx) * fy, fx * fy};
            const int32_t ni[4] = {ci, ci + 1, ci, ci + 1};
            const int32_t nj[4] = {cj, cj, cj + 1, cj + 1};
            for (int32_t pp = 0; pp < P; ++pp) {
                uint32_t acc = 0;
                for (int32_t c = 0; c < 4; ++c) {
                    if (ni[c] < 0 || ni[c] >= n || nj[c] < 0 || nj[c] >= n) continue;
                    const int64_t cn = (int64_t)nj[c] * n + ni[c];
                    acc += W[c] * (uint32_t)src[cn * P + pp];
                }
                const uint16_t val = (uint16_t)((acc + (1u << 15)) >> 16);
                if (val != phi[node * P + pp]) {
                    phi[node * P + pp] = val;
                    changed = 1;
                }
            }
        }
        ++passes;
        if (!changed) break;
    }
    free(prev);
    for (int64_t node = 0; node < N; ++node) {
        int32_t best = -1;
        uint32_t bv = 0;
        for (int32_t pp = 0; pp < P; ++pp) {
            if (phi[node * P + pp] > bv) { bv = phi[node * P + pp]; best = pp; }
        }
        label[node] = (int16_t)best;
    }
    return passes;
}

/* One Jacobi sweep of the per-patch computation with state constraints at the interfaces
 * (the first-order patchy method, Section 2): a node of patch p reads every grid value that
 * belongs to another patch as v_out, i.e. its patch is solved as if it were the whole
 * domain. Nodes with label -1 form a group of their own. */
double or_sweep_independent(const or_problem* p, const int16_t* label, const double* v_in, double* v_out,
                            int32_t n_threads) {
    const int64_t N = (int64_t)p->n * p->n;
    double resid = 0.0;
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for reduction(max : resid) num_threads(n_threads) schedule(dynamic, 64)
    for (int64_t node = 0; node < N; ++node) {
        const uint8_t cls = p->node_class[node];
        if (cls != OR_FREE) {
            v_out[node] = or_fixed_value(p, cls);
            continue;
        }
        /* the node's view of the grid: own-patch values, v_out elsewhere */
        const double beta = or_beta(p);
        double best = INFINITY;
        for (int32_t m = 0; m < p->n_controls; ++m) {
            const double rho = or_rho_at(p, (int32_t)node, m);
            double y[8];
            const int32_t K = or_feet(p, (int32_t)(node % p->n), (int32_t)(node / p->n), m, y);
            double mean = 0.0, lam0 = 0.0, lam1 = 0.0;
            for (int32_t k = 0; k < K; ++k) {
                int32_t idx[4];
                double w[4];
                if (!or_interp_weights(p, y[2 * k], y[2 * k + 1], idx, w)) {
                    mean += p->v_out;
                    lam1 += p->v_out;
                    continue;
                }
                for (int32_t c = 0; c < 4; ++c) {
                    const double val = label[idx[c]] == label[node] ? v_in[idx[c]] : p->v_out;
                    mean += w[c] * val;
                    if (idx[c] == node) lam0 += w[c];
                    else lam1 += w[c] * val;
                }
            }
            mean /= K;
            lam0 /= K;
            lam1 /= K;
            const double q = p->scheme == OR_SL3 ? (beta * lam1 + rho) / (1.0 - beta * lam0) : beta * mean + rho;
            if (q < best) best = q;
        }
        v_out[node] = best;
        const double d = fabs(best - v_in[node]);
        if (d > resid) resid = d;
    }
    return resid;
}
