/*
 * fse_oracle.c -- plain FP64 CPU oracle for Frequency Selective Extrapolation
 * (FSE) with the line-scan, the optimized (Algorithm 1) and a refined
 * (sample-count) processing order.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU implementation: every quantity here is
 * recomputed from the paper's definitions, slowly and directly.
 *
 * What it computes (Section 2 of the paper, with the readings listed below):
 *   - the extrapolation area L = block b plus a frame of d samples, M x N,
 *     with subareas A (known), R (reconstructed), B_i (lost in b),
 *     B_o (lost outside b);
 *   - the weighting function of Eq. (2): rho^dist on A, delta*rho^dist on R,
 *     0 on B_i and B_o, dist measured from ((M-1)/2, (N-1)/2);
 *   - the model of Eq. (1), g = sum_{k in K} c_k phi_k, built greedily: in
 *     every iteration one DFT basis function (Section 4) is selected and its
 *     expansion coefficient estimated with orthogonality deficiency
 *     compensation factor gamma (Section 4);
 *   - the samples of B_i taken from the model;
 *   - the block processing orders of Section 2 (line scan) and Section 3
 *     (Algorithm 1 with Eq. (3)), and the refined criterion that Section 3
 *     suggests without specifying it (counting the unknown samples of the
 *     neighbouring blocks instead of the neighbouring blocks with losses).
 *
 * Readings of points the paper leaves open (each is a design decision, not a
 * statement of the paper):
 *   - selection: the weighted least-squares projection of the residual r on
 *     phi_k is p_k = sum(w r conj(phi_k)) / sum(w |phi_k|^2) = P[k] / W0,
 *     because |phi_k| = 1; adding gamma*p_k*phi_k lowers the weighted residual
 *     energy by (2 gamma - gamma^2)|P[k]|^2 / W0, so the selected index is
 *     argmax |P[k]|^2 and the coefficient update is gamma * P[u] / W0;
 *   - ties in the argmax go to the smallest row-major index k1*NF + k2;
 *   - the basis is phi_k[m,n] = exp(+j 2 pi (k1 m / MF + k2 n / NF)) on an
 *     MF x NF grid with L placed at its top-left corner; the output is Re g;
 *   - exactly K iterations; an index may be selected again;
 *   - an area without support (W0 == 0) is filled with a constant;
 *   - neighbours are the 8-neighbourhood; the rim penalty is the number of
 *     missing 8-neighbours (so +3 at a margin block, +5 at a corner block);
 *   - N_min is the smallest non-negative N (the printed Eq. (3) reads 0 as
 *     soon as one block is done, which would stall the loop);
 *   - every block of a wave reads the image as it was at the start of the
 *     wave (snapshot semantics);
 *   - refined order: N(b) = sum over the 8 neighbours of the number of lost,
 *     not yet extrapolated samples in that neighbour, where a neighbour cell
 *     outside the image counts as a whole block of unknown samples (the
 *     sample-count analogue of the +3 / +5 rim penalty); waves are formed
 *     exactly as in Algorithm 1 (smallest non-negative N, raster order, no
 *     two adjacent blocks), and after a wave every pending neighbour of a
 *     finished block loses that block's unknown samples from its N.  When
 *     every lost block is lost entirely, N is B_h*B_w times Algorithm 1's N
 *     and both orders coincide.
 *
 * Projections are explicit separable spatial-domain sums, recomputed from
 * the spatial residual in every iteration.  No FFT, no spectral shortcut.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* Sample classes inside an extrapolation area. */
enum { CLS_A = 0, CLS_R = 1, CLS_BI = 2, CLS_BO = 3, CLS_OUT = 4 };
/* Per-sample image state. */
enum { ST_KNOWN = 0, ST_PENDING = 1, ST_RECON = 2 };

typedef struct {
  int32_t block_w, block_h;   /* block size (samples) */
  int32_t border_d;           /* frame width d around the block */
  int32_t fft_w, fft_h;       /* basis grid NF (columns) x MF (rows) */
  double rho;                 /* weighting decay */
  double delta;               /* reconstructed-area attenuation */
  double gamma;               /* orthogonality deficiency compensation */
  int32_t iterations;         /* K */
  int32_t order;              /* 0 = optimized (Algorithm 1), 1 = line scan, 2 = refined */
  double empty_fill;          /* value for an area without support */
  int32_t tie_largest;        /* test switch: ties go to the largest index */
  int32_t frame_off_m;        /* test switch: row offset of L in the grid */
  int32_t frame_off_n;        /* test switch: column offset of L in the grid */
  int32_t nthreads;           /* worker threads for the blocks of one wave */
  int32_t grid_off_x;         /* block grid shift: block column j covers */
  int32_t grid_off_y;         /*   x in [j*block_w - grid_off_x, +block_w) */
} oracle_params;

/* cos/sin(2 pi t / n) for t = 0..n-1, built so that the table is exactly
 * symmetric: c[n-t] == c[t] and s[n-t] == -s[t]. */
static void twiddles(int n, double *c, double *s) {
  for (int t = 0; t <= n / 2; ++t) {
    double a = 2.0 * OR_PI * (double)t / (double)n;
    c[t] = cos(a);
    s[t] = sin(a);
  }
  for (int t = n / 2 + 1; t < n; ++t) {
    c[t] = c[n - t];
    s[t] = -s[n - t];
  }
  /* pin exact zeros at the quarter points when they exist */
  if (n % 4 == 0) {
    c[n / 4] = 0.0;
    c[3 * n / 4] = 0.0;
  }
  if (n % 2 == 0) s[n / 2] = 0.0;
}

static int imod(long a, int n) {
  long r = a % n;
  return (int)(r < 0 ? r + n : r);
}

/* Weighting function of Eq. (2) for one sample. */
static double weight_of(const oracle_params *p, int M, int N, int m, int n, int cls) {
  double dm = (double)m - 0.5 * (double)(M - 1);
  double dn = (double)n - 0.5 * (double)(N - 1);
  double radial = pow(p->rho, sqrt(dm * dm + dn * dn));
  if (cls == CLS_A) return radial;
  if (cls == CLS_R) return p->delta * radial;
  return 0.0;
}

/*
 * Weighted DFT of (w * r) over the MF x NF basis grid, as explicit separable
 * sums: P[k1][k2] = sum_m e^{-j2pi k1 (m+om)/MF} sum_n w r e^{-j2pi k2 (n+on)/NF}.
 * q is scratch of size M*NF complex.
 */
static void weighted_dft(int M, int N, int MF, int NF, int om, int on,
                         const double *w, const double *rr, const double *ri,
                         const double *cm, const double *sm,
                         const double *cn, const double *sn,
                         double *qr, double *qi, double *pr, double *pi) {
  for (int m = 0; m < M; ++m) {
    for (int k2 = 0; k2 < NF; ++k2) {
      double ar = 0.0, ai = 0.0;
      for (int n = 0; n < N; ++n) {
        double wv = w[m * N + n];
        double xr = wv * rr[m * N + n], xi = wv * ri[m * N + n];
        int t = imod((long)k2 * (n + on), NF);
        /* (xr + j xi) * (cos - j sin) */
        ar += xr * cn[t] + xi * sn[t];
        ai += xi * cn[t] - xr * sn[t];
      }
      qr[m * NF + k2] = ar;
      qi[m * NF + k2] = ai;
    }
  }
  for (int k1 = 0; k1 < MF; ++k1) {
    for (int k2 = 0; k2 < NF; ++k2) {
      double ar = 0.0, ai = 0.0;
      for (int m = 0; m < M; ++m) {
        int t = imod((long)k1 * (m + om), MF);
        double xr = qr[m * NF + k2], xi = qi[m * NF + k2];
        ar += xr * cm[t] + xi * sm[t];
        ai += xi * cm[t] - xr * sm[t];
      }
      pr[k1 * NF + k2] = ar;
      pi[k1 * NF + k2] = ai;
    }
  }
}

/* e^{+j2pi (k1 (m+om)/MF + k2 (n+on)/NF)} */
static void basis_at(int k1, int k2, int m, int n, int MF, int NF, int om, int on,
                     const double *cm, const double *sm, const double *cn,
                     const double *sn, double *br, double *bi) {
  int t1 = imod((long)k1 * (m + om), MF);
  int t2 = imod((long)k2 * (n + on), NF);
  double c1 = cm[t1], s1 = sm[t1], c2 = cn[t2], s2 = sn[t2];
  *br = c1 * c2 - s1 * s2;
  *bi = s1 * c2 + c1 * s2;
}

/*
 * One block: FSE over an extrapolation area (Section 2, Eq. (1) and (2)).
 *   f      : M*N sample values of L (values on B_i/B_o/outside are ignored)
 *   f_im   : M*N imaginary parts (nullable; a complex test signal)
 *   cls    : M*N classes (CLS_*)
 *   g_out  : M*N, Re of the final model over all of L (nullable)
 *   u_out  : K selected indices k1*NF + k2 (nullable)
 *   dc_out : 2K, (re, im) coefficient increments (nullable)
 *   e_out  : K+1 weighted residual energies sum w |r|^2, before iteration 1
 *            and after every iteration (nullable)
 *   spec_out: 2*MF*NF, P of the residual after `spec_iter` iterations
 *            (nullable; spec_iter in 0..K)
 * Returns 0, or 1 if L has no support (W0 == 0); then g_out = empty_fill.
 */
int oracle_block(const oracle_params *p, int M, int N, const double *f,
                 const double *f_im, const uint8_t *cls, double *g_out, int32_t *u_out,
                 double *dc_out, double *e_out, double *w0_out,
                 double *spec_out, int spec_iter) {
  const int MF = p->fft_h, NF = p->fft_w, K = p->iterations;
  const int om = p->frame_off_m, on = p->frame_off_n;
  double *w = (double *)malloc(sizeof(double) * M * N);
  double *rr = (double *)malloc(sizeof(double) * M * N);
  double *ri = (double *)malloc(sizeof(double) * M * N);
  double *qr = (double *)malloc(sizeof(double) * M * NF);
  double *qi = (double *)malloc(sizeof(double) * M * NF);
  double *pr = (double *)malloc(sizeof(double) * MF * NF);
  double *pi = (double *)malloc(sizeof(double) * MF * NF);
  double *cr = (double *)calloc((size_t)MF * NF, sizeof(double));
  double *ci = (double *)calloc((size_t)MF * NF, sizeof(double));
  double *cm = (double *)malloc(sizeof(double) * MF);
  double *sm = (double *)malloc(sizeof(double) * MF);
  double *cn = (double *)malloc(sizeof(double) * NF);
  double *sn = (double *)malloc(sizeof(double) * NF);
  twiddles(MF, cm, sm);
  twiddles(NF, cn, sn);

  double W0 = 0.0;
  for (int m = 0; m < M; ++m)
    for (int n = 0; n < N; ++n) {
      int c = cls[m * N + n];
      double wv = weight_of(p, M, N, m, n, c);
      w[m * N + n] = wv;
      W0 += wv;
      int sup = (c == CLS_A || c == CLS_R);
      rr[m * N + n] = sup ? f[m * N + n] : 0.0;
      ri[m * N + n] = (sup && f_im) ? f_im[m * N + n] : 0.0;
    }
  if (w0_out) *w0_out = W0;

  int rc = 0;
  if (W0 == 0.0) {
    if (g_out)
      for (int i = 0; i < M * N; ++i) g_out[i] = p->empty_fill;
    if (u_out)
      for (int i = 0; i < K; ++i) u_out[i] = -1;
    if (dc_out)
      for (int i = 0; i < 2 * K; ++i) dc_out[i] = 0.0;
    if (e_out)
      for (int i = 0; i <= K; ++i) e_out[i] = 0.0;
    rc = 1;
    goto done;
  }

  if (e_out) {
    double e = 0.0;
    for (int i = 0; i < M * N; ++i) e += w[i] * (rr[i] * rr[i] + ri[i] * ri[i]);
    e_out[0] = e;
  }
  for (int it = 0; it < K; ++it) {
    weighted_dft(M, N, MF, NF, om, on, w, rr, ri, cm, sm, cn, sn, qr, qi, pr, pi);
    if (spec_out && spec_iter == it)
      for (int k = 0; k < MF * NF; ++k) {
        spec_out[2 * k] = pr[k];
        spec_out[2 * k + 1] = pi[k];
      }
    /* selection: largest |P|^2 */
    int u = 0;
    double best = -1.0;
    for (int k = 0; k < MF * NF; ++k) {
      double e = pr[k] * pr[k] + pi[k] * pi[k];
      if (e > best || (p->tie_largest && e == best)) {
        best = e;
        u = k;
      }
    }
    /* coefficient estimate with orthogonality deficiency compensation */
    double dcr = p->gamma * pr[u] / W0, dci = p->gamma * pi[u] / W0;
    cr[u] += dcr;
    ci[u] += dci;
    if (u_out) u_out[it] = u;
    if (dc_out) {
      dc_out[2 * it] = dcr;
      dc_out[2 * it + 1] = dci;
    }
    /* residual update in the spatial domain: r -= dc * phi_u */
    int u1 = u / NF, u2 = u % NF;
    double e = 0.0;
    for (int m = 0; m < M; ++m)
      for (int n = 0; n < N; ++n) {
        double br, bi;
        basis_at(u1, u2, m, n, MF, NF, om, on, cm, sm, cn, sn, &br, &bi);
        double *a = &rr[m * N + n], *b = &ri[m * N + n];
        double nr = *a - (dcr * br - dci * bi);
        double ni = *b - (dcr * bi + dci * br);
        *a = nr;
        *b = ni;
        e += w[m * N + n] * (nr * nr + ni * ni);
      }
    if (e_out) e_out[it + 1] = e;
  }
  if (spec_out && spec_iter == K) {
    weighted_dft(M, N, MF, NF, om, on, w, rr, ri, cm, sm, cn, sn, qr, qi, pr, pi);
    for (int k = 0; k < MF * NF; ++k) {
      spec_out[2 * k] = pr[k];
      spec_out[2 * k + 1] = pi[k];
    }
  }
  /* the model of Eq. (1) over L; the caller keeps the samples of B_i */
  if (g_out) {
    for (int m = 0; m < M; ++m)
      for (int n = 0; n < N; ++n) {
        double acc = 0.0;
        for (int k = 0; k < MF * NF; ++k) {
          if (cr[k] == 0.0 && ci[k] == 0.0) continue;
          double br, bi;
          basis_at(k / NF, k % NF, m, n, MF, NF, om, on, cm, sm, cn, sn, &br, &bi);
          acc += cr[k] * br - ci[k] * bi;
        }
        g_out[m * N + n] = acc;
      }
  }
done:
  free(w); free(rr); free(ri); free(qr); free(qi); free(pr); free(pi);
  free(cr); free(ci); free(cm); free(sm); free(cn); free(sn);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Processing order (Section 2 line scan; Section 3, Algorithm 1, Eq. (3))  */
/* ------------------------------------------------------------------------ */

/*
 * The two orders of Section 3 share one loop, written from the section's
 * description rather than from Algorithm 1's incremental bookkeeping: before
 * every wave the count N(b) of each pending block is recomputed from its
 * definition, the smallest non-negative count is taken, the pending blocks
 * with that count are scanned in raster order and a block joins the wave
 * unless one of its 8 neighbours has already joined; the blocks of the wave
 * are then marked extrapolated.
 *
 * weight[b] is what a pending neighbour b contributes to a count, `outside`
 * what a neighbour position outside the image contributes.  Algorithm 1:
 * weight 1 for a block with lost samples and outside = 1 (a missing
 * neighbour counts as not extrapolated, which is the +3 margin and +5 corner
 * rule).  Refined order: weight = the block's lost samples and outside = a
 * whole block's samples.
 */
static long neighbour_count(int hb, int wb, const long *weight, const uint8_t *pending,
                            long outside, int i, int j) {
  long n = 0;
  for (int di = -1; di <= 1; ++di)
    for (int dj = -1; dj <= 1; ++dj) {
      if (!di && !dj) continue;
      int y = i + di, x = j + dj;
      if (y < 0 || y >= hb || x < 0 || x >= wb)
        n += outside;
      else if (pending[y * wb + x])
        n += weight[y * wb + x];
    }
  return n;
}

static int waves_by_count(int hb, int wb, const long *weight, long outside,
                          int32_t *wave_of, int32_t *order_out) {
  int nb = hb * wb, nwaves = 0, pos = 0;
  uint8_t *pending = (uint8_t *)malloc((size_t)nb);
  uint8_t *in_s = (uint8_t *)malloc((size_t)nb);
  long *cnt = (long *)malloc(sizeof(long) * nb);
  for (int b = 0; b < nb; ++b) {
    wave_of[b] = -1;
    pending[b] = weight[b] > 0;
  }
  for (;;) {
    long nmin = -1;
    for (int i = 0; i < hb; ++i)
      for (int j = 0; j < wb; ++j) {
        int b = i * wb + j;
        if (!pending[b]) continue;
        cnt[b] = neighbour_count(hb, wb, weight, pending, outside, i, j);
        if (nmin < 0 || cnt[b] < nmin) nmin = cnt[b];
      }
    if (nmin < 0) break;  /* nothing left to extrapolate */
    memset(in_s, 0, (size_t)nb);
    for (int i = 0; i < hb; ++i)
      for (int j = 0; j < wb; ++j) {
        int b = i * wb + j;
        if (!pending[b] || cnt[b] != nmin) continue;
        int touches = 0;
        for (int di = -1; di <= 1; ++di)
          for (int dj = -1; dj <= 1; ++dj) {
            int y = i + di, x = j + dj;
            if ((di || dj) && y >= 0 && y < hb && x >= 0 && x < wb && in_s[y * wb + x])
              touches = 1;
          }
        if (touches) continue;
        in_s[b] = 1;
        wave_of[b] = nwaves;
        if (order_out) order_out[pos] = b;
        ++pos;
      }
    for (int b = 0; b < nb; ++b)
      if (in_s[b]) pending[b] = 0;
    ++nwaves;
  }
  free(pending);
  free(in_s);
  free(cnt);
  return nwaves;
}

/*
 * lost[hb*wb]: nonzero if the block has samples to extrapolate.
 * wave_of[hb*wb] (out): wave index of each lost block, -1 for the others.
 * order_out[hb*wb] (out, nullable): lost blocks in processing order (waves in
 * sequence, raster order inside a wave).
 * order: 1 = line scan (Section 2), otherwise Algorithm 1 (Section 3).
 * Returns the number of waves.
 */
int oracle_schedule(int hb, int wb, const uint8_t *lost, int order,
                    int32_t *wave_of, int32_t *order_out) {
  if (hb <= 0 || wb <= 0) return 0;
  int nb = hb * wb;
  if (order == 1) {
    int nwaves = 0, pos = 0;
    for (int b = 0; b < nb; ++b) {
      wave_of[b] = -1;
      if (lost[b]) {
        wave_of[b] = nwaves++;
        if (order_out) order_out[pos++] = b;
      }
    }
    return nwaves;
  }
  long *weight = (long *)malloc(sizeof(long) * nb);
  for (int b = 0; b < nb; ++b) weight[b] = lost[b] ? 1 : 0;
  int nw = waves_by_count(hb, wb, weight, 1, wave_of, order_out);
  free(weight);
  return nw;
}

/*
 * Refined order (the criterion Section 3 mentions as an alternative).
 * unknown[hb*wb]: lost samples of each block (0 = nothing to extrapolate);
 * outside: the count a neighbour cell outside the image contributes (a whole
 * block, B_h*B_w).  Outputs as oracle_schedule.  Returns the number of waves.
 */
int oracle_schedule_refined(int hb, int wb, const int32_t *unknown, int outside,
                            int32_t *wave_of, int32_t *order_out) {
  if (hb <= 0 || wb <= 0) return 0;
  int nb = hb * wb;
  long *weight = (long *)malloc(sizeof(long) * nb);
  for (int b = 0; b < nb; ++b) weight[b] = unknown[b] > 0 ? unknown[b] : 0;
  int nw = waves_by_count(hb, wb, weight, outside, wave_of, order_out);
  free(weight);
  return nw;
}

/* ------------------------------------------------------------------------ */
/* Whole image                                                              */
/* ------------------------------------------------------------------------ */

/* Extract L of block (bi, bj) from a snapshot: values and classes. */
static void extract_area(const oracle_params *p, int H, int W, const double *img,
                         const uint8_t *state, int bi, int bj, int M, int N,
                         double *f, uint8_t *cls) {
  int y0 = bi * p->block_h - p->grid_off_y, x0 = bj * p->block_w - p->grid_off_x;
  int y1 = y0 + p->block_h < H ? y0 + p->block_h : H;
  int x1 = x0 + p->block_w < W ? x0 + p->block_w : W;
  for (int m = 0; m < M; ++m)
    for (int n = 0; n < N; ++n) {
      int y = y0 - p->border_d + m, x = x0 - p->border_d + n;
      int c;
      double v = 0.0;
      if (y < 0 || y >= H || x < 0 || x >= W) {
        c = CLS_OUT;
      } else {
        int s = state[y * W + x];
        v = img[y * W + x];
        if (s == ST_KNOWN) c = CLS_A;
        else if (s == ST_RECON) c = CLS_R;
        else c = (y >= y0 && y < y1 && x >= x0 && x < x1) ? CLS_BI : CLS_BO;
      }
      f[m * N + n] = v;
      cls[m * N + n] = (uint8_t)c;
    }
}

/*
 * Conceal one image.
 *   img     : H*W sample values (lost samples ignored)
 *   lost    : H*W, nonzero = lost
 *   out     : H*W result (known samples copied, lost samples extrapolated)
 *   wave_of : hb*wb (out, nullable) wave index per block, -1 if not lost
 *   trace_u : hb*wb*K (out, nullable) selected indices per block
 *   trace_dc: hb*wb*2K (out, nullable) coefficient increments per block
 * Returns the number of waves, or -1 on invalid parameters.
 */
int oracle_conceal(const oracle_params *p, int H, int W, const double *img,
                   const uint8_t *lost, double *out, int32_t *wave_of,
                   int32_t *trace_u, double *trace_dc) {
  if (H <= 0 || W <= 0 || p->block_w <= 0 || p->block_h <= 0 || p->border_d < 0 ||
      p->grid_off_x < 0 || p->grid_off_x >= p->block_w || p->grid_off_y < 0 ||
      p->grid_off_y >= p->block_h || p->order < 0 || p->order > 2)
    return -1;
  const int M = p->block_h + 2 * p->border_d, N = p->block_w + 2 * p->border_d;
  if (M > p->fft_h || N > p->fft_w) return -1;
  const int hb = (H + p->grid_off_y + p->block_h - 1) / p->block_h;
  const int wb = (W + p->grid_off_x + p->block_w - 1) / p->block_w;
  const int nb = hb * wb, K = p->iterations;
  uint8_t *blost = (uint8_t *)calloc((size_t)nb, 1);
  int32_t *bcnt = (int32_t *)calloc((size_t)nb, sizeof(int32_t));  /* lost samples per block */
  uint8_t *state = (uint8_t *)malloc((size_t)H * W);
  uint8_t *snap_state = (uint8_t *)malloc((size_t)H * W);
  double *snap = (double *)malloc(sizeof(double) * H * W);
  int32_t *wv = (int32_t *)malloc(sizeof(int32_t) * nb);
  int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * nb);
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int l = lost[y * W + x] != 0;
      state[y * W + x] = l ? ST_PENDING : ST_KNOWN;
      out[y * W + x] = l ? 0.0 : img[y * W + x];
      if (l) {
        int b = ((y + p->grid_off_y) / p->block_h) * wb + (x + p->grid_off_x) / p->block_w;
        blost[b] = 1;
        bcnt[b] += 1;
      }
    }
  int nw = p->order == 2 ? oracle_schedule_refined(hb, wb, bcnt, p->block_h * p->block_w, wv, ord)
                         : oracle_schedule(hb, wb, blost, p->order, wv, ord);
  if (wave_of) memcpy(wave_of, wv, sizeof(int32_t) * nb);
  int pos = 0, nlost = 0;
  for (int b = 0; b < nb; ++b) nlost += blost[b] != 0;
  for (int wave = 0; wave < nw; ++wave) {
    int start = pos;
    while (pos < nlost && wv[ord[pos]] == wave) ++pos;
    memcpy(snap, out, sizeof(double) * H * W);
    memcpy(snap_state, state, (size_t)H * W);
    int count = pos - start;
#ifdef _OPENMP
    int nt = p->nthreads > 0 ? p->nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int q = 0; q < count; ++q) {
      int b = ord[start + q];
      int bi = b / wb, bj = b % wb;
      double *f = (double *)malloc(sizeof(double) * M * N);
      double *g = (double *)malloc(sizeof(double) * M * N);
      uint8_t *cls = (uint8_t *)malloc((size_t)M * N);
      extract_area(p, H, W, snap, snap_state, bi, bj, M, N, f, cls);
      oracle_block(p, M, N, f, NULL, cls, g,
                   trace_u ? trace_u + (size_t)b * K : NULL,
                   trace_dc ? trace_dc + (size_t)b * 2 * K : NULL,
                   NULL, NULL, NULL, -1);
      /* insert the model samples of B_i; they become reconstructed */
      for (int m = 0; m < M; ++m)
        for (int n = 0; n < N; ++n)
          if (cls[m * N + n] == CLS_BI) {
            int y = bi * p->block_h - p->grid_off_y - p->border_d + m;
            int x = bj * p->block_w - p->grid_off_x - p->border_d + n;
            out[y * W + x] = g[m * N + n];
            state[y * W + x] = ST_RECON;
          }
      free(f); free(g); free(cls);
    }
  }
  free(blost); free(bcnt); free(state); free(snap_state); free(snap); free(wv); free(ord);
  return nw;
}

/* Extract the area of one block from a given working image and state map
 * (used to feed a block the exact input another implementation saw). */
void oracle_extract_area(const oracle_params *p, int H, int W, const double *img,
                         const uint8_t *state, int bi, int bj, double *f,
                         uint8_t *cls) {
  const int M = p->block_h + 2 * p->border_d, N = p->block_w + 2 * p->border_d;
  extract_area(p, H, W, img, state, bi, bj, M, N, f, cls);
}
