/*
 * CPU checker: exact discrete k-eigenvalue power iteration by transport sweeps.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call
 * this file; it exists to produce the expected values that the device
 * solver is checked against.
 *
 * Everything here follows the paper's statement of the discrete problem:
 *  - the vertex diamond-difference cell equation (Section 2.1, eq.
 *    Discretized_kNTE): for cell (k,j,i) and direction l,
 *      mu/(4dx) * sum_{k',j'} (psi[k',j',i] - psi[k',j',i-1])
 *    + eta/(4dy) * sum_{k',i'} (psi[k',j,i'] - psi[k',j-1,i'])
 *    + xi/(4dz)  * sum_{j',i'} (psi[k,j',i'] - psi[k-1,j',i'])
 *    + sigma_t/8 * sum over the 8 vertices of psi
 *    = q[g, cell],
 *    with the isotropic source
 *      q[g, cell] = 1/8 * sum_g' (sigma_s[g<-g'] + chi[g] nu_sigma_f[g'] / k)
 *                       * sum_l' w_l' * sum over the 8 vertices of psi[g', l'];
 *  - vacuum boundary equations psi = 0 on the incoming faces of each
 *    direction (appendix, eq. discreteBCs);
 *  - the solve of H by a sweep (the forward substitution described for the
 *    comparison code in the section on reference values): cells are visited
 *    in the direction of travel so that 7 of the 8 vertices of each cell are
 *    known and the cell equation gives the remaining (outgoing) vertex;
 *  - the power iteration of eq. k_eff_fixed_points: one sweep of every
 *    (group, direction) per step with the source of the previous iterate,
 *    k_{t+1} = k_t * sum(F psi_{t+1}) / sum(F psi_t).
 *
 * A checker-only reflective mode (incoming face value = value of the mirror
 * direction at the same node, taken from the previous iterate; x mirror has
 * priority on edges, then y, then z) gives the infinite-medium closed form.
 *
 * Layouts: psi[g][l][k][j][i] with node counts nz, ny, nx (i fastest);
 * cell material mat[ck][cj][ci] over (nz-1)(ny-1)(nx-1) cells;
 * sigma_t[m][g], sigma_s[m][g][gp] (gp -> g), nu_sigma_f[m][g], chi[g].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t G, L, nz, ny, nx;
  double hz, hy, hx;
  const double *mu, *eta, *xi, *w;      /* [L] */
  const int64_t *mat;                   /* [(nz-1)(ny-1)(nx-1)] */
  const double *sigma_t;                /* [Mat][G] */
  const double *sigma_s;                /* [Mat][G][G] */
  const double *nu_sigma_f;             /* [Mat][G] */
  const double *chi;                    /* [G] */
  int64_t reflective[3];                /* per axis z, y, x: 0 vacuum, 1 reflective */
} dd_problem;

#define NODE(p, k, j, i) (((k) * (p)->ny + (j)) * (p)->nx + (i))

static int64_t nodes(const dd_problem *p) { return p->nz * p->ny * p->nx; }
static int64_t cells(const dd_problem *p) { return (p->nz - 1) * (p->ny - 1) * (p->nx - 1); }

/* phi8[g][cell] = sum_l w_l * (sum of psi over the 8 vertices of the cell). */
void dd_phi8(const dd_problem *p, const double *psi, double *phi8) {
  const int64_t N = nodes(p), C = cells(p);
  const int64_t Kc = p->nz - 1, Jc = p->ny - 1, Ic = p->nx - 1;
  for (int64_t g = 0; g < p->G; ++g) {
    double *out = phi8 + g * C;
    memset(out, 0, sizeof(double) * C);
    for (int64_t l = 0; l < p->L; ++l) {
      const double *ps = psi + (g * p->L + l) * N;
      const double wl = p->w[l];
      for (int64_t ck = 0; ck < Kc; ++ck)
        for (int64_t cj = 0; cj < Jc; ++cj)
          for (int64_t ci = 0; ci < Ic; ++ci) {
            double s = 0.0;
            for (int dk = 0; dk < 2; ++dk)
              for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di) s += ps[NODE(p, ck + dk, cj + dj, ci + di)];
            out[(ck * Jc + cj) * Ic + ci] += wl * s;
          }
    }
  }
}

/* q[g][cell] = 1/8 sum_g' (sigma_s[g<-g'] + chi[g] nu_sigma_f[g'] * inv_k) phi8[g'][cell]. */
void dd_source(const dd_problem *p, const double *phi8, double inv_k, double *q) {
  const int64_t C = cells(p), G = p->G;
  for (int64_t c = 0; c < C; ++c) {
    const int64_t m = p->mat[c];
    for (int64_t g = 0; g < G; ++g) {
      double s = 0.0;
      for (int64_t gp = 0; gp < G; ++gp) {
        const double coef = p->sigma_s[(m * G + g) * G + gp] + p->chi[g] * p->nu_sigma_f[m * G + gp] * inv_k;
        s += coef * phi8[gp * C + c];
      }
      q[g * C + c] = 0.125 * s;
    }
  }
}

/* Sum of all entries of F psi: every (g, l) row block of a cell carries
 * 1/8 chi[g] sum_g' nu_sigma_f[g'] phi8[g'][cell]; boundary rows carry 0. */
double dd_fission_total(const dd_problem *p, const double *phi8) {
  const int64_t C = cells(p), G = p->G;
  double total = 0.0;
  for (int64_t c = 0; c < C; ++c) {
    const int64_t m = p->mat[c];
    double f = 0.0;
    for (int64_t gp = 0; gp < G; ++gp) f += p->nu_sigma_f[m * G + gp] * phi8[gp * C + c];
    for (int64_t g = 0; g < G; ++g) total += (double)p->L * 0.125 * p->chi[g] * f;
  }
  return total;
}

static int64_t mirror(const dd_problem *p, int64_t l, int axis_bit) {
  /* octant o = bx + 2 by + 4 bz, directions grouped per octant */
  const int64_t per = p->L / 8;
  const int64_t o = l / per, m = l % per;
  return (o ^ axis_bit) * per + m;
}

/* One sweep of direction l of group g: solve the cell equations for the
 * source q (isotropic, [cell]) with incoming-face values from the boundary
 * rule.  psi_prev is used only for reflective faces. */
static void sweep_one(const dd_problem *p, int64_t g, int64_t l, const double *q,
                      const double *psi_prev, double *out) {
  const int64_t N = nodes(p);
  const int64_t Kc = p->nz - 1, Jc = p->ny - 1, Ic = p->nx - 1;
  const double mu = p->mu[l], eta = p->eta[l], xi = p->xi[l];
  const int64_t i_in = mu > 0 ? 0 : p->nx - 1;
  const int64_t j_in = eta > 0 ? 0 : p->ny - 1;
  const int64_t k_in = xi > 0 ? 0 : p->nz - 1;
  const double *prev_x = psi_prev + (g * p->L + mirror(p, l, 1)) * N;
  const double *prev_y = psi_prev + (g * p->L + mirror(p, l, 2)) * N;
  const double *prev_z = psi_prev + (g * p->L + mirror(p, l, 4)) * N;
  /* incoming faces */
  for (int64_t k = 0; k < p->nz; ++k)
    for (int64_t j = 0; j < p->ny; ++j)
      for (int64_t i = 0; i < p->nx; ++i) {
        const int64_t n = NODE(p, k, j, i);
        double v = 0.0;
        if (i == i_in) v = p->reflective[2] ? prev_x[n] : 0.0;
        else if (j == j_in) v = p->reflective[1] ? prev_y[n] : 0.0;
        else if (k == k_in) v = p->reflective[0] ? prev_z[n] : 0.0;
        out[n] = v;
      }
  const double A = mu / (4.0 * p->hx), B = eta / (4.0 * p->hy), Cz = xi / (4.0 * p->hz);
  for (int64_t a = 0; a < Kc; ++a) {
    const int64_t ck = xi > 0 ? 1 + a : Kc - a;          /* cell index 1..Kc */
    for (int64_t b = 0; b < Jc; ++b) {
      const int64_t cj = eta > 0 ? 1 + b : Jc - b;
      for (int64_t c = 0; c < Ic; ++c) {
        const int64_t ci = mu > 0 ? 1 + c : Ic - c;
        const int64_t cell = ((ck - 1) * Jc + (cj - 1)) * Ic + (ci - 1);
        const int64_t m = p->mat[cell];
        const double D = p->sigma_t[m * p->G + g] / 8.0;
        const int64_t ok = xi > 0 ? ck : ck - 1;
        const int64_t oj = eta > 0 ? cj : cj - 1;
        const int64_t oi = mu > 0 ? ci : ci - 1;
        out[NODE(p, ok, oj, oi)] = 0.0;
        double lhs = 0.0;
        for (int64_t kk = ck - 1; kk <= ck; ++kk)
          for (int64_t jj = cj - 1; jj <= cj; ++jj)
            lhs += A * (out[NODE(p, kk, jj, ci)] - out[NODE(p, kk, jj, ci - 1)]);
        for (int64_t kk = ck - 1; kk <= ck; ++kk)
          for (int64_t ii = ci - 1; ii <= ci; ++ii)
            lhs += B * (out[NODE(p, kk, cj, ii)] - out[NODE(p, kk, cj - 1, ii)]);
        for (int64_t jj = cj - 1; jj <= cj; ++jj)
          for (int64_t ii = ci - 1; ii <= ci; ++ii)
            lhs += Cz * (out[NODE(p, ck, jj, ii)] - out[NODE(p, ck - 1, jj, ii)]);
        double s8 = 0.0;
        for (int64_t kk = ck - 1; kk <= ck; ++kk)
          for (int64_t jj = cj - 1; jj <= cj; ++jj)
            for (int64_t ii = ci - 1; ii <= ci; ++ii) s8 += out[NODE(p, kk, jj, ii)];
        lhs += D * s8;
        const double diag = fabs(A) + fabs(B) + fabs(Cz) + D;
        out[NODE(p, ok, oj, oi)] = (q[cell] - lhs) / diag;
      }
    }
  }
}

/* psi_out = H^{-1} (source rows q): one sweep of every (g, l). */
void dd_sweep(const dd_problem *p, const double *q, const double *psi_prev, double *psi_out) {
  const int64_t N = nodes(p), C = cells(p);
#pragma omp parallel for collapse(2) schedule(dynamic)
  for (int64_t g = 0; g < p->G; ++g)
    for (int64_t l = 0; l < p->L; ++l)
      sweep_one(p, g, l, q + g * C, psi_prev, psi_out + (g * p->L + l) * N);
}

/* Power iteration of eq. k_eff_fixed_points.  psi (in/out) holds psi_0 on
 * entry and the last iterate on exit, scaled to unit 2-norm.  k_hist[0..steps]
 * receives k_0..k_steps.  Returns the number of steps taken. */
int64_t dd_power_iteration(const dd_problem *p, double *psi, double k0, double tol_k,
                           int64_t max_steps, double *k_hist) {
  const int64_t N = nodes(p), C = cells(p), T = p->G * p->L * N;
  double *phi8 = (double *)malloc(sizeof(double) * p->G * C);
  double *q = (double *)malloc(sizeof(double) * p->G * C);
  double *next = (double *)malloc(sizeof(double) * T);
  double k = k0;
  k_hist[0] = k;
  dd_phi8(p, psi, phi8);
  double fis = dd_fission_total(p, phi8);
  int64_t step = 0;
  while (step < max_steps) {
    dd_source(p, phi8, 1.0 / k, q);
    dd_sweep(p, q, psi, next);
    dd_phi8(p, next, phi8);
    const double fis_next = dd_fission_total(p, phi8);
    const double k_next = k * fis_next / fis;
    double nrm = 0.0;
    for (int64_t t = 0; t < T; ++t) nrm += next[t] * next[t];
    nrm = sqrt(nrm);
    for (int64_t t = 0; t < T; ++t) psi[t] = next[t] / nrm;
    for (int64_t c = 0; c < p->G * C; ++c) phi8[c] /= nrm;
    fis = fis_next / nrm;
    ++step;
    k_hist[step] = k_next;
    const double dk = fabs(k_next - k);
    k = k_next;
    if (dk < tol_k) break;
  }
  free(phi8);
  free(q);
  free(next);
  return step;
}

/* One power step from (psi, k): writes the unnormalized iterate and returns k_next. */
double dd_power_step(const dd_problem *p, const double *psi, double k, double *psi_next) {
  const int64_t C = cells(p);
  double *phi8 = (double *)malloc(sizeof(double) * p->G * C);
  double *q = (double *)malloc(sizeof(double) * p->G * C);
  dd_phi8(p, psi, phi8);
  const double fis = dd_fission_total(p, phi8);
  dd_source(p, phi8, 1.0 / k, q);
  dd_sweep(p, q, psi, psi_next);
  dd_phi8(p, psi_next, phi8);
  const double fis_next = dd_fission_total(p, phi8);
  free(phi8);
  free(q);
  return k * fis_next / fis;
}
