/*
 * fse_oracle3d.c -- plain FP64 CPU oracle for three-dimensional Frequency
 * Selective Extrapolation of a video volume (frames x rows x columns).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite may load this library.  It
 * shares no code, header, table or helper with the GPU implementation (nor
 * with the two-dimensional oracle in fse_oracle.c): every quantity is
 * recomputed from the definitions, slowly and directly.
 *
 * The paper develops its processing order for two-dimensional signals and
 * states, in its conclusion, that the method extends to higher-dimensional
 * signals through three-dimensional FSE, where parallel execution matters
 * even more because of the cost.  Nothing else about the 3-D form is given;
 * the reading implemented here carries every 2-D definition over one more
 * dimension:
 *   - the volume is divided into blocks of B_t x B_h x B_w samples; a block
 *     holding lost samples is extrapolated from its area L = the block plus
 *     d_t frames before and after and d samples around it in each frame,
 *     M_t x M x N samples, nominal geometry at the volume's faces (samples
 *     outside the volume weigh 0);
 *   - weighting function (Eq. (2) in three dimensions): rho^dist on known
 *     samples, delta rho^dist on reconstructed ones, 0 on lost ones, with
 *     dist the Euclidean distance of (t, m, n) from the centre
 *     ((M_t-1)/2, (M-1)/2, (N-1)/2);
 *   - basis: phi_k[t,m,n] = exp(+j 2 pi (k1 t / F_t + k2 m / F_h + k3 n / F_w))
 *     on an F_t x F_h x F_w grid with L at its first corner; the model of
 *     Eq. (1) is generated greedily exactly as in two dimensions (select
 *     argmax |P[k]|^2 of the weighted DFT of the residual, add
 *     gamma P[u] / W0, exactly K iterations, ties to the smallest index
 *     (k1 F_h + k2) F_w + k3); the output is the real part;
 *   - processing order: Algorithm 1 over the 26-neighbourhood of a block in
 *     the block grid (frames, rows, columns): N(b) = number of lost,
 *     not yet extrapolated 26-neighbours + the number of missing
 *     26-neighbours at the volume's faces (the 2-D rim rule, 26 - number of
 *     neighbours inside the grid); a wave takes, in raster order (frame, row,
 *     column), every pending block with the smallest non-negative N that has
 *     no 26-neighbour in the wave; N is recounted from this definition before
 *     every wave; line scan = lost blocks in raster order, one per wave;
 *   - every block of a wave reads the volume as it was at the start of the
 *     wave (snapshot semantics).
 * With one frame (M_t = F_t = 1, blocks one frame deep) every sum below runs
 * exactly the two-dimensional oracle's arithmetic, so the result equals the
 * 2-D oracle's bit for bit (pinned in the tests).
 *
 * Projections are explicit separable spatial-domain sums recomputed from the
 * spatial residual in every iteration.  No FFT, no spectral shortcut.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR3_PI 3.14159265358979323846

enum { C3_A = 0, C3_R = 1, C3_BI = 2, C3_BO = 3, C3_OUT = 4 };
enum { S3_KNOWN = 0, S3_PENDING = 1, S3_RECON = 2 };

typedef struct {
  int32_t block_t, block_h, block_w; /* block size (frames, rows, columns) */
  int32_t border_t, border_d;        /* d_t frames, d samples around the block */
  int32_t fft_t, fft_h, fft_w;       /* basis grid F_t x F_h x F_w */
  double rho, delta, gamma;
  int32_t iterations;                /* K */
  int32_t order;                     /* 0 = Algorithm 1 (26-neighbourhood), 1 = line scan */
  double empty_fill;
  int32_t nthreads;
} oracle3_params;

/* cos/sin(2 pi t / n), t = 0..n-1, exactly symmetric (as in fse_oracle.c,
 * written again here: the two oracles share nothing). */
static void tw3(int n, double *c, double *s) {
  for (int t = 0; t <= n / 2; ++t) {
    double a = 2.0 * OR3_PI * (double)t / (double)n;
    c[t] = cos(a);
    s[t] = sin(a);
  }
  for (int t = n / 2 + 1; t < n; ++t) {
    c[t] = c[n - t];
    s[t] = -s[n - t];
  }
  if (n % 4 == 0) {
    c[n / 4] = 0.0;
    c[3 * n / 4] = 0.0;
  }
  if (n % 2 == 0) s[n / 2] = 0.0;
}

static int md3(long a, int n) {
  long r = a % n;
  return (int)(r < 0 ? r + n : r);
}

static double weight3(const oracle3_params *p, int Mt, int M, int N, int t, int m, int n,
                      int cls) {
  double dt = (double)t - 0.5 * (double)(Mt - 1);
  double dm = (double)m - 0.5 * (double)(M - 1);
  double dn = (double)n - 0.5 * (double)(N - 1);
  double radial = pow(p->rho, sqrt(dt * dt + dm * dm + dn * dn));
  if (cls == C3_A) return radial;
  if (cls == C3_R) return p->delta * radial;
  return 0.0;
}

/* P[k1][k2][k3] = sum_t e^{-j2pi k1 t/Ft} sum_m e^{-j2pi k2 m/Fh}
 *                 sum_n w r e^{-j2pi k3 n/Fw}, three passes of explicit sums. */
static void wdft3(int Mt, int M, int N, int Ft, int Fh, int Fw, const double *w,
                  const double *rr, const double *ri, const double *ct, const double *st,
                  const double *ch, const double *sh, const double *cw, const double *sw,
                  double *q1r, double *q1i, double *q2r, double *q2i, double *pr, double *pi) {
  for (int t = 0; t < Mt; ++t)
    for (int m = 0; m < M; ++m)
      for (int k3 = 0; k3 < Fw; ++k3) {
        double ar = 0.0, ai = 0.0;
        for (int n = 0; n < N; ++n) {
          size_t i = ((size_t)t * M + m) * N + n;
          double wv = w[i];
          double xr = wv * rr[i], xi = wv * ri[i];
          int a = md3((long)k3 * n, Fw);
          ar += xr * cw[a] + xi * sw[a];
          ai += xi * cw[a] - xr * sw[a];
        }
        q1r[((size_t)t * M + m) * Fw + k3] = ar;
        q1i[((size_t)t * M + m) * Fw + k3] = ai;
      }
  for (int t = 0; t < Mt; ++t)
    for (int k2 = 0; k2 < Fh; ++k2)
      for (int k3 = 0; k3 < Fw; ++k3) {
        double ar = 0.0, ai = 0.0;
        for (int m = 0; m < M; ++m) {
          int a = md3((long)k2 * m, Fh);
          double xr = q1r[((size_t)t * M + m) * Fw + k3], xi = q1i[((size_t)t * M + m) * Fw + k3];
          ar += xr * ch[a] + xi * sh[a];
          ai += xi * ch[a] - xr * sh[a];
        }
        q2r[((size_t)t * Fh + k2) * Fw + k3] = ar;
        q2i[((size_t)t * Fh + k2) * Fw + k3] = ai;
      }
  for (int k1 = 0; k1 < Ft; ++k1)
    for (int k2 = 0; k2 < Fh; ++k2)
      for (int k3 = 0; k3 < Fw; ++k3) {
        double ar = 0.0, ai = 0.0;
        for (int t = 0; t < Mt; ++t) {
          int a = md3((long)k1 * t, Ft);
          double xr = q2r[((size_t)t * Fh + k2) * Fw + k3], xi = q2i[((size_t)t * Fh + k2) * Fw + k3];
          ar += xr * ct[a] + xi * st[a];
          ai += xi * ct[a] - xr * st[a];
        }
        pr[((size_t)k1 * Fh + k2) * Fw + k3] = ar;
        pi[((size_t)k1 * Fh + k2) * Fw + k3] = ai;
      }
}

/* e^{+j2pi (k1 t/Ft + k2 m/Fh + k3 n/Fw)}: the (m, n) factor first, then t */
static void basis3(int k1, int k2, int k3, int t, int m, int n, int Ft, int Fh, int Fw,
                   const double *ct, const double *st, const double *ch, const double *sh,
                   const double *cw, const double *sw, double *br, double *bi) {
  int a2 = md3((long)k2 * m, Fh), a3 = md3((long)k3 * n, Fw), a1 = md3((long)k1 * t, Ft);
  double c2 = ch[a2], s2 = sh[a2], c3 = cw[a3], s3 = sw[a3];
  double xr = c2 * c3 - s2 * s3;
  double xi = s2 * c3 + c2 * s3;
  double c1 = ct[a1], s1 = st[a1];
  *br = xr * c1 - xi * s1;
  *bi = xi * c1 + xr * s1;
}

/*
 * One block: FSE over a 3-D area of Mt x M x N samples.
 *   f, f_im : sample values (imaginary part nullable: a complex test signal)
 *   cls     : classes C3_*
 *   g_out   : Re of the model over L (nullable)
 *   u_out   : K selected indices (k1 Fh + k2) Fw + k3; dc_out: 2K increments
 *   e_out   : K+1 weighted residual energies; w0_out: sum of weights
 *   spec_out: 2 Ft Fh Fw, P of the residual after spec_iter iterations
 * Returns 0, or 1 if L has no support (then g_out = empty_fill).
 */
int oracle3_block(const oracle3_params *p, int Mt, int M, int N, const double *f,
                  const double *f_im, const uint8_t *cls, double *g_out, int32_t *u_out,
                  double *dc_out, double *e_out, double *w0_out, double *spec_out,
                  int spec_iter) {
  const int Ft = p->fft_t, Fh = p->fft_h, Fw = p->fft_w, K = p->iterations;
  const size_t L = (size_t)Mt * M * N, F = (size_t)Ft * Fh * Fw;
  double *w = (double *)malloc(sizeof(double) * L);
  double *rr = (double *)malloc(sizeof(double) * L);
  double *ri = (double *)malloc(sizeof(double) * L);
  double *q1r = (double *)malloc(sizeof(double) * Mt * M * Fw);
  double *q1i = (double *)malloc(sizeof(double) * Mt * M * Fw);
  double *q2r = (double *)malloc(sizeof(double) * Mt * Fh * Fw);
  double *q2i = (double *)malloc(sizeof(double) * Mt * Fh * Fw);
  double *pr = (double *)malloc(sizeof(double) * F);
  double *pi = (double *)malloc(sizeof(double) * F);
  double *cr = (double *)calloc(F, sizeof(double));
  double *ci = (double *)calloc(F, sizeof(double));
  double *ct = (double *)malloc(sizeof(double) * Ft), *st = (double *)malloc(sizeof(double) * Ft);
  double *ch = (double *)malloc(sizeof(double) * Fh), *sh = (double *)malloc(sizeof(double) * Fh);
  double *cw = (double *)malloc(sizeof(double) * Fw), *sw = (double *)malloc(sizeof(double) * Fw);
  tw3(Ft, ct, st);
  tw3(Fh, ch, sh);
  tw3(Fw, cw, sw);

  double W0 = 0.0;
  for (int t = 0; t < Mt; ++t)
    for (int m = 0; m < M; ++m)
      for (int n = 0; n < N; ++n) {
        size_t i = ((size_t)t * M + m) * N + n;
        int c = cls[i];
        double wv = weight3(p, Mt, M, N, t, m, n, c);
        w[i] = wv;
        W0 += wv;
        int sup = (c == C3_A || c == C3_R);
        rr[i] = sup ? f[i] : 0.0;
        ri[i] = (sup && f_im) ? f_im[i] : 0.0;
      }
  if (w0_out) *w0_out = W0;
  int rc = 0;
  if (W0 == 0.0) {
    if (g_out)
      for (size_t i = 0; i < L; ++i) g_out[i] = p->empty_fill;
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
    for (size_t i = 0; i < L; ++i) e += w[i] * (rr[i] * rr[i] + ri[i] * ri[i]);
    e_out[0] = e;
  }
  for (int it = 0; it < K; ++it) {
    wdft3(Mt, M, N, Ft, Fh, Fw, w, rr, ri, ct, st, ch, sh, cw, sw, q1r, q1i, q2r, q2i, pr, pi);
    if (spec_out && spec_iter == it)
      for (size_t k = 0; k < F; ++k) {
        spec_out[2 * k] = pr[k];
        spec_out[2 * k + 1] = pi[k];
      }
    int u = 0;
    double best = -1.0;
    for (size_t k = 0; k < F; ++k) {
      double e = pr[k] * pr[k] + pi[k] * pi[k];
      if (e > best) {
        best = e;
        u = (int)k;
      }
    }
    double dcr = p->gamma * pr[u] / W0, dci = p->gamma * pi[u] / W0;
    cr[u] += dcr;
    ci[u] += dci;
    if (u_out) u_out[it] = u;
    if (dc_out) {
      dc_out[2 * it] = dcr;
      dc_out[2 * it + 1] = dci;
    }
    int u1 = u / (Fh * Fw), u2 = (u / Fw) % Fh, u3 = u % Fw;
    double e = 0.0;
    for (int t = 0; t < Mt; ++t)
      for (int m = 0; m < M; ++m)
        for (int n = 0; n < N; ++n) {
          size_t i = ((size_t)t * M + m) * N + n;
          double br, bi;
          basis3(u1, u2, u3, t, m, n, Ft, Fh, Fw, ct, st, ch, sh, cw, sw, &br, &bi);
          double nr = rr[i] - (dcr * br - dci * bi);
          double ni = ri[i] - (dcr * bi + dci * br);
          rr[i] = nr;
          ri[i] = ni;
          e += w[i] * (nr * nr + ni * ni);
        }
    if (e_out) e_out[it + 1] = e;
  }
  if (spec_out && spec_iter == K) {
    wdft3(Mt, M, N, Ft, Fh, Fw, w, rr, ri, ct, st, ch, sh, cw, sw, q1r, q1i, q2r, q2i, pr, pi);
    for (size_t k = 0; k < F; ++k) {
      spec_out[2 * k] = pr[k];
      spec_out[2 * k + 1] = pi[k];
    }
  }
  if (g_out) {
    for (int t = 0; t < Mt; ++t)
      for (int m = 0; m < M; ++m)
        for (int n = 0; n < N; ++n) {
          double acc = 0.0;
          for (size_t k = 0; k < F; ++k) {
            if (cr[k] == 0.0 && ci[k] == 0.0) continue;
            int k1 = (int)(k / ((size_t)Fh * Fw)), k2 = (int)((k / Fw) % Fh), k3 = (int)(k % Fw);
            double br, bi;
            basis3(k1, k2, k3, t, m, n, Ft, Fh, Fw, ct, st, ch, sh, cw, sw, &br, &bi);
            acc += cr[k] * br - ci[k] * bi;
          }
          g_out[((size_t)t * M + m) * N + n] = acc;
        }
  }
done:
  free(w); free(rr); free(ri); free(q1r); free(q1i); free(q2r); free(q2i); free(pr); free(pi);
  free(cr); free(ci); free(ct); free(st); free(ch); free(sh); free(cw); free(sw);
  return rc;
}

/*
 * Processing order over a tb x hb x wb block grid (lost[b] nonzero = the
 * block holds lost samples).  wave_of[b] = wave index (-1 if not lost), seq =
 * lost blocks in processing order.  Returns the number of waves.
 */
int oracle3_schedule(int tb, int hb, int wb, const uint8_t *lost, int order, int32_t *wave_of,
                     int32_t *seq) {
  if (tb <= 0 || hb <= 0 || wb <= 0) return 0;
  const int nb = tb * hb * wb;
  int nlost = 0, pos = 0;
  for (int b = 0; b < nb; ++b) {
    wave_of[b] = -1;
    nlost += lost[b] != 0;
  }
  if (order == 1) {
    int w = 0;
    for (int b = 0; b < nb; ++b)
      if (lost[b]) {
        wave_of[b] = w++;
        seq[pos++] = b;
      }
    return w;
  }
  uint8_t *pending = (uint8_t *)malloc((size_t)nb);
  uint8_t *in_wave = (uint8_t *)malloc((size_t)nb);
  int *cnt = (int *)malloc(sizeof(int) * (size_t)nb);
  for (int b = 0; b < nb; ++b) pending[b] = lost[b] != 0;
  int waves = 0;
  while (pos < nlost) {
    /* N(b) from its definition: pending 26-neighbours + missing ones */
    int nmin = -1;
    for (int b = 0; b < nb; ++b) {
      cnt[b] = -1;
      if (!pending[b]) continue;
      int t = b / (hb * wb), i = (b / wb) % hb, j = b % wb, c = 0;
      for (int a = -1; a <= 1; ++a)
        for (int di = -1; di <= 1; ++di)
          for (int dj = -1; dj <= 1; ++dj) {
            if (!a && !di && !dj) continue;
            int tt = t + a, ii = i + di, jj = j + dj;
            if (tt < 0 || tt >= tb || ii < 0 || ii >= hb || jj < 0 || jj >= wb)
              c += 1; /* missing neighbour: counts as not extrapolated */
            else if (pending[(tt * hb + ii) * wb + jj])
              c += 1;
          }
      cnt[b] = c;
      if (nmin < 0 || c < nmin) nmin = c;
    }
    memset(in_wave, 0, (size_t)nb);
    for (int b = 0; b < nb; ++b) {
      if (cnt[b] != nmin) continue;
      int t = b / (hb * wb), i = (b / wb) % hb, j = b % wb, clash = 0;
      for (int a = -1; a <= 1 && !clash; ++a)
        for (int di = -1; di <= 1 && !clash; ++di)
          for (int dj = -1; dj <= 1 && !clash; ++dj) {
            int tt = t + a, ii = i + di, jj = j + dj;
            if ((a || di || dj) && tt >= 0 && tt < tb && ii >= 0 && ii < hb && jj >= 0 &&
                jj < wb && in_wave[(tt * hb + ii) * wb + jj])
              clash = 1;
          }
      if (clash) continue;
      in_wave[b] = 1;
      wave_of[b] = waves;
      seq[pos++] = b;
    }
    for (int b = 0; b < nb; ++b)
      if (in_wave[b]) pending[b] = 0;
    ++waves;
  }
  free(pending);
  free(in_wave);
  free(cnt);
  return waves;
}

/* Area of block (bt, bi, bj) from a snapshot of the volume: values, classes. */
static void area3(const oracle3_params *p, int T, int H, int W, const double *vol,
                  const uint8_t *state, int bt, int bi, int bj, int Mt, int M, int N, double *f,
                  uint8_t *cls) {
  int t0 = bt * p->block_t, y0 = bi * p->block_h, x0 = bj * p->block_w;
  int t1 = t0 + p->block_t < T ? t0 + p->block_t : T;
  int y1 = y0 + p->block_h < H ? y0 + p->block_h : H;
  int x1 = x0 + p->block_w < W ? x0 + p->block_w : W;
  for (int t = 0; t < Mt; ++t)
    for (int m = 0; m < M; ++m)
      for (int n = 0; n < N; ++n) {
        int z = t0 - p->border_t + t, y = y0 - p->border_d + m, x = x0 - p->border_d + n;
        size_t i = ((size_t)t * M + m) * N + n;
        int c;
        double v = 0.0;
        if (z < 0 || z >= T || y < 0 || y >= H || x < 0 || x >= W) {
          c = C3_OUT;
        } else {
          size_t q = ((size_t)z * H + y) * W + x;
          int s = state[q];
          v = vol[q];
          if (s == S3_KNOWN) c = C3_A;
          else if (s == S3_RECON) c = C3_R;
          else c = (z >= t0 && z < t1 && y >= y0 && y < y1 && x >= x0 && x < x1) ? C3_BI : C3_BO;
        }
        f[i] = v;
        cls[i] = (uint8_t)c;
      }
}

void oracle3_extract_area(const oracle3_params *p, int T, int H, int W, const double *vol,
                          const uint8_t *state, int bt, int bi, int bj, double *f,
                          uint8_t *cls) {
  area3(p, T, H, W, vol, state, bt, bi, bj, p->block_t + 2 * p->border_t,
        p->block_h + 2 * p->border_d, p->block_w + 2 * p->border_d, f, cls);
}

/*
 * Conceal a volume of T frames of H x W samples (frame-major).  out receives
 * the volume with the lost samples extrapolated; wave_of (nullable) the wave
 * of every block.  Returns the number of waves, -1 on invalid parameters.
 */
int oracle3_conceal(const oracle3_params *p, int T, int H, int W, const double *vol,
                    const uint8_t *lost, double *out, int32_t *wave_of) {
  if (T <= 0 || H <= 0 || W <= 0 || p->block_t <= 0 || p->block_h <= 0 || p->block_w <= 0 ||
      p->border_t < 0 || p->border_d < 0 || p->order < 0 || p->order > 1)
    return -1;
  const int Mt = p->block_t + 2 * p->border_t, M = p->block_h + 2 * p->border_d,
            N = p->block_w + 2 * p->border_d;
  if (Mt > p->fft_t || M > p->fft_h || N > p->fft_w) return -1;
  const int tb = (T + p->block_t - 1) / p->block_t, hb = (H + p->block_h - 1) / p->block_h,
            wb = (W + p->block_w - 1) / p->block_w;
  const int nb = tb * hb * wb;
  const size_t V = (size_t)T * H * W, L = (size_t)Mt * M * N;
  uint8_t *blost = (uint8_t *)calloc((size_t)nb, 1);
  uint8_t *state = (uint8_t *)malloc(V), *snap_state = (uint8_t *)malloc(V);
  double *snap = (double *)malloc(sizeof(double) * V);
  int32_t *wv = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
  int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
  for (int z = 0; z < T; ++z)
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        size_t q = ((size_t)z * H + y) * W + x;
        int l = lost[q] != 0;
        state[q] = l ? S3_PENDING : S3_KNOWN;
        out[q] = l ? 0.0 : vol[q];
        if (l) blost[((z / p->block_t) * hb + y / p->block_h) * wb + x / p->block_w] = 1;
      }
  int nw = oracle3_schedule(tb, hb, wb, blost, p->order, wv, ord);
  if (wave_of) memcpy(wave_of, wv, sizeof(int32_t) * nb);
  int nlost = 0, pos = 0;
  for (int b = 0; b < nb; ++b) nlost += blost[b] != 0;
  for (int wave = 0; wave < nw; ++wave) {
    int start = pos;
    while (pos < nlost && wv[ord[pos]] == wave) ++pos;
    memcpy(snap, out, sizeof(double) * V);
    memcpy(snap_state, state, V);
    int count = pos - start;
#ifdef _OPENMP
    int nt = p->nthreads > 0 ? p->nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int q = 0; q < count; ++q) {
      int b = ord[start + q];
      int bt = b / (hb * wb), bi = (b / wb) % hb, bj = b % wb;
      double *f = (double *)malloc(sizeof(double) * L), *g = (double *)malloc(sizeof(double) * L);
      uint8_t *cls = (uint8_t *)malloc(L);
      area3(p, T, H, W, snap, snap_state, bt, bi, bj, Mt, M, N, f, cls);
      oracle3_block(p, Mt, M, N, f, NULL, cls, g, NULL, NULL, NULL, NULL, NULL, -1);
      for (int t = 0; t < Mt; ++t)
        for (int m = 0; m < M; ++m)
          for (int n = 0; n < N; ++n)
            if (cls[((size_t)t * M + m) * N + n] == C3_BI) {
              int z = bt * p->block_t - p->border_t + t, y = bi * p->block_h - p->border_d + m,
                  x = bj * p->block_w - p->border_d + n;
              size_t i = ((size_t)z * H + y) * W + x;
              out[i] = g[((size_t)t * M + m) * N + n];
              state[i] = S3_RECON;
            }
      free(f); free(g); free(cls);
    }
  }
  free(blost); free(state); free(snap_state); free(snap); free(wv); free(ord);
  return nw;
}
