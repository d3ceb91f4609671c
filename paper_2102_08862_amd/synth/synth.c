/*
 * Seeded synthetic TPC time-frame generator.
 *
 * Produces clusters in the native TPC coordinates the tracker consumes
 * (pad row, pad-direction y, drift time), one cluster per pad row a helix
 * crosses, for Pb-Pb-like continuous-readout frames: collisions at 50 kHz
 * spread uniformly over the frame, so that a 10 ms frame holds ~500
 * overlapping collisions (the paper's time frames of ~10 ms, Sec. 1).
 *
 * This module is the input generator only. It holds the detector geometry
 * and the forward simulation of helices; it holds none of the tracking
 * method (neighbour finding, cellular automaton, Kalman fit).
 *
 * Geometry (the paper gives none; readings chosen for this build):
 *   - 36 sectors of 20 degrees, 0..17 on the A side (z > 0), 18..35 on the
 *     C side (z < 0); sector s is centred at alpha = ((s mod 18) + 0.5)*20 deg.
 *   - Sector-local frame: X along the sector centre, Y perpendicular.
 *   - 152 pad rows at X = x_r = (float)(85 + r*160/151) cm, half width
 *     x_r * tan(10 deg).
 *   - Drift: L = 250 cm, v_d = 2.58 cm/us; time is stored in cm of drift:
 *     t = v_d * t_collision + (L - |z|). Single-sector workloads use t = z.
 *   - Curvature kappa = d(phi)/d(arc) = -kB * q/pT with kB = 2.99792458e-3*Bz.
 *
 * Randomness: counter-based splitmix64 streams (Steele, Lea, Flood 2014)
 * keyed by (seed, stream id), so results do not depend on thread count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYN_NROWS 152
#define SYN_NSECT 36
#define SYN_PI 3.14159265358979323846
#define SYN_DEG (SYN_PI / 180.0)

/* ------------------------------------------------------------------ RNG */
typedef struct { uint64_t s; } syn_rng;

static uint64_t syn_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static syn_rng syn_stream(uint64_t seed, uint64_t id) {
    syn_rng r;
    r.s = syn_mix(seed * 0x9E3779B97F4A7C15ull + syn_mix(id + 0x632BE59BD9B4E019ull));
    return r;
}
static uint64_t syn_next(syn_rng *r) {
    r->s += 0x9E3779B97F4A7C15ull;
    return syn_mix(r->s);
}
static double syn_unif(syn_rng *r) { return (double)(syn_next(r) >> 11) * 0x1.0p-53; }
static double syn_normal(syn_rng *r) {
    double u1 = 1.0 - syn_unif(r); /* (0, 1] */
    double u2 = syn_unif(r);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * SYN_PI * u2);
}
static double syn_exp(syn_rng *r, double mean) { return -mean * log(1.0 - syn_unif(r)); }

/* ------------------------------------------------------------- geometry */
static double syn_row_x(int r) { return (double)(float)(85.0 + r * 160.0 / 151.0); }
static double syn_half_width(int r) { return (double)(float)(syn_row_x(r) * tan(10.0 * SYN_DEG)); }
static double syn_alpha(int s) { return ((s % 18) + 0.5) * 20.0 * SYN_DEG; }

void synth_geometry(int32_t n_rows, float *row_x, float *half_width) {
    for (int r = 0; r < n_rows && r < SYN_NROWS; r++) {
        row_x[r] = (float)syn_row_x(r);
        half_width[r] = (float)syn_half_width(r);
    }
}

/* -------------------------------------------------------------- params */
typedef struct {
    uint64_t seed;
    int32_t single_sector;  /* 1: one sector, t = z, phi within the sector */
    int32_t n_collisions;   /* collisions in the frame */
    int32_t fixed_mult;     /* >0: exactly this many tracks per collision */
    double frame_us;        /* frame length (us) */
    double bz;              /* tesla */
    double sigma_y, sigma_t;
    double noise_frac;      /* noise clusters per signal cluster, per sector */
    double quant;           /* cluster values rounded to multiples of this; 0 = off */
    double mult_mean, mult_max;
    double pt_min, pt_mean; /* pT = pt_min + Exp(pt_mean) */
    double eta_max;
    double zv_sigma;
    double vdrift, drift_len;
    int32_t n_threads;
} synth_params;

typedef struct { uint8_t sector, row; float y, t; int32_t label; } syn_rec;
typedef struct { syn_rec *v; int64_t n, cap; } syn_buf;

static void syn_push(syn_buf *b, syn_rec r) {
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 4096;
        b->v = (syn_rec *)realloc(b->v, (size_t)b->cap * sizeof(syn_rec));
    }
    b->v[b->n++] = r;
}

typedef struct {
    double q, pt, phi0, tgl, zv, tcoll_us, kappa, eta;
    int32_t collision;
} syn_track;

typedef struct {
    int64_t n[SYN_NSECT];
    uint8_t *row[SYN_NSECT];
    float *y[SYN_NSECT], *t[SYN_NSECT];
    int32_t *label[SYN_NSECT];
    int64_t n_tracks;
    syn_track *tracks;
    double t_lo, t_hi;
} synth_frame;

static double syn_quant(double v, double q) { return q > 0 ? nearbyint(v / q) * q : v; }

/* Rising-X crossing of the helix with the row line X = x in the local frame
 * of azimuth alpha, on the outgoing half turn. Returns 1 and fills Y and the
 * transverse arc length when it exists. */
static int syn_cross(const syn_track *tr, double alpha, double x, double *Y, double *arc) {
    double k = tr->kappa;
    double pl = tr->phi0 - alpha;
    double sp = sin(pl);
    double u = sp + k * x;
    if (!(fabs(u) <= 1.0)) return 0;
    double psi = asin(u);
    double d = psi - pl;
    /* smallest arc >= 0 with pl + k*arc == psi (mod 2 pi) */
    double twopi = 2.0 * SYN_PI;
    double a;
    if (k > 0) {
        a = fmod(d, twopi); if (a < 0) a += twopi;
        a /= k;
    } else {
        a = fmod(-d, twopi); if (a < 0) a += twopi;
        a /= -k;
    }
    if (a > SYN_PI / fabs(k)) return 0;
    /* cos(pl) - cos(psi) = 2 sin((psi+pl)/2) sin((psi-pl)/2), with psi - pl = k*a */
    double dpsi = k * a;
    *Y = 2.0 * sin(pl + 0.5 * dpsi) * sin(0.5 * dpsi) / k;
    *arc = a;
    return 1;
}

typedef struct {
    const synth_params *p;
    syn_track *tracks;
    int64_t *first_track;   /* per collision */
    syn_buf *bufs;          /* per collision */
    int32_t n_coll;
    int32_t next;
    pthread_mutex_t mu;
} syn_job;

static void syn_gen_collision(const synth_params *p, syn_track *tracks, int64_t first, int64_t ntr,
                              int32_t c, syn_buf *out) {
    syn_rng rng = syn_stream(p->seed, 1 + (uint64_t)c);
    double kB = 2.99792458e-3 * p->bz;
    double rho_min = syn_row_x(0);
    double rho_max = syn_row_x(SYN_NROWS - 1) / cos(10.0 * SYN_DEG);
    for (int64_t j = 0; j < ntr; j++) {
        syn_track *tr = &tracks[first + j];
        tr->q = (syn_unif(&rng) < 0.5) ? -1.0 : 1.0;
        tr->pt = p->pt_min + syn_exp(&rng, p->pt_mean);
        tr->eta = -p->eta_max + 2.0 * p->eta_max * syn_unif(&rng);
        tr->tgl = sinh(tr->eta);
        if (p->single_sector)
            tr->phi0 = syn_alpha(0) + (-10.0 + 20.0 * syn_unif(&rng)) * SYN_DEG;
        else
            tr->phi0 = 2.0 * SYN_PI * syn_unif(&rng);
        tr->kappa = -kB * tr->q / tr->pt;
        tr->collision = c;
        double k = tr->kappa;
        double ak = fabs(k);
        double two_r = 2.0 / ak;
        if (two_r < rho_min) continue;
        double rmax = rho_max < two_r ? rho_max : two_r;
        double la = 2.0 * asin(fmin(1.0, rho_min * ak / 2.0)) / ak;
        double lb = 2.0 * asin(fmin(1.0, rmax * ak / 2.0)) / ak;
        double th_a = tr->phi0 + 0.5 * k * la, th_b = tr->phi0 + 0.5 * k * lb;
        double th_lo = fmin(th_a, th_b) - 1.0 * SYN_DEG, th_hi = fmax(th_a, th_b) + 1.0 * SYN_DEG;
        int na = p->single_sector ? 1 : 18;
        for (int a = 0; a < na; a++) {
            double al = syn_alpha(a);
            /* angular overlap of [al-10, al+10] with [th_lo, th_hi] modulo 2 pi */
            double lo = al - 10.0 * SYN_DEG, hi = al + 10.0 * SYN_DEG;
            int hit = 0;
            for (int w = -2; w <= 2 && !hit; w++) {
                double o = w * 2.0 * SYN_PI;
                if (hi + o >= th_lo && lo + o <= th_hi) hit = 1;
            }
            if (!hit) continue;
            for (int r = 0; r < SYN_NROWS; r++) {
                double x = syn_row_x(r), Y, arc;
                if (!syn_cross(tr, al, x, &Y, &arc)) continue;
                if (fabs(Y) > syn_half_width(r)) continue;
                double z = tr->zv + tr->tgl * arc;
                if (fabs(z) > p->drift_len) continue;
                int sector;
                double t;
                if (p->single_sector) {
                    sector = 0;
                    t = z;
                } else {
                    if (z == 0.0) continue;
                    sector = (z > 0) ? a : 18 + a;
                    t = p->vdrift * tr->tcoll_us + (p->drift_len - fabs(z));
                }
                double ys = Y + p->sigma_y * syn_normal(&rng);
                double ts = t + p->sigma_t * syn_normal(&rng);
                syn_rec rec;
                rec.sector = (uint8_t)sector;
                rec.row = (uint8_t)r;
                rec.y = (float)syn_quant(ys, p->quant);
                rec.t = (float)syn_quant(ts, p->quant);
                rec.label = (int32_t)(first + j);
                syn_push(out, rec);
            }
        }
    }
}

static void *syn_worker(void *arg) {
    syn_job *jb = (syn_job *)arg;
    for (;;) {
        pthread_mutex_lock(&jb->mu);
        int32_t c = jb->next++;
        pthread_mutex_unlock(&jb->mu);
        if (c >= jb->n_coll) break;
        int64_t first = jb->first_track[c];
        int64_t ntr = jb->first_track[c + 1] - first;
        syn_gen_collision(jb->p, jb->tracks, first, ntr, c, &jb->bufs[c]);
    }
    return NULL;
}

typedef struct {
    const synth_params *p;
    synth_frame *f;
    int32_t next;
    pthread_mutex_t mu;
} syn_noise_job;

static void syn_noise_sector(const synth_params *p, synth_frame *f, int s) {
    syn_rng rng = syn_stream(p->seed, 1000000ull + (uint64_t)s);
    int64_t nsig = f->n[s];
    int64_t nn = (int64_t)llround(p->noise_frac * (double)nsig);
    int64_t n = nsig + nn;
    f->row[s] = (uint8_t *)realloc(f->row[s], (size_t)(n ? n : 1));
    f->y[s] = (float *)realloc(f->y[s], (size_t)(n ? n : 1) * 4);
    f->t[s] = (float *)realloc(f->t[s], (size_t)(n ? n : 1) * 4);
    f->label[s] = (int32_t *)realloc(f->label[s], (size_t)(n ? n : 1) * 4);
    for (int64_t i = nsig; i < n; i++) {
        int r = (int)(syn_unif(&rng) * SYN_NROWS);
        if (r >= SYN_NROWS) r = SYN_NROWS - 1;
        double hw = syn_half_width(r);
        f->row[s][i] = (uint8_t)r;
        f->y[s][i] = (float)syn_quant(-hw + 2.0 * hw * syn_unif(&rng), p->quant);
        f->t[s][i] = (float)syn_quant(f->t_lo + (f->t_hi - f->t_lo) * syn_unif(&rng), p->quant);
        f->label[s][i] = -1;
    }
    f->n[s] = n;
    /* Fisher-Yates shuffle of the sector's clusters */
    for (int64_t i = n - 1; i > 0; i--) {
        int64_t j = (int64_t)(syn_unif(&rng) * (double)(i + 1));
        if (j > i) j = i;
        uint8_t tr = f->row[s][i]; f->row[s][i] = f->row[s][j]; f->row[s][j] = tr;
        float ty = f->y[s][i]; f->y[s][i] = f->y[s][j]; f->y[s][j] = ty;
        float tt = f->t[s][i]; f->t[s][i] = f->t[s][j]; f->t[s][j] = tt;
        int32_t tl = f->label[s][i]; f->label[s][i] = f->label[s][j]; f->label[s][j] = tl;
    }
}

static void *syn_noise_worker(void *arg) {
    syn_noise_job *jb = (syn_noise_job *)arg;
    for (;;) {
        pthread_mutex_lock(&jb->mu);
        int32_t s = jb->next++;
        pthread_mutex_unlock(&jb->mu);
        if (s >= SYN_NSECT) break;
        syn_noise_sector(jb->p, jb->f, s);
    }
    return NULL;
}

void synth_params_default(synth_params *p) {
    memset(p, 0, sizeof(*p));
    p->seed = 1;
    p->single_sector = 0;
    p->n_collisions = 50;
    p->fixed_mult = 0;
    p->frame_us = 1000.0;
    p->bz = 0.5;
    p->sigma_y = 0.1;
    p->sigma_t = 0.1;
    p->noise_frac = 0.05;
    p->quant = 1.0 / 512.0;
    p->mult_mean = 2000.0;
    p->mult_max = 15000.0;
    p->pt_min = 0.1;
    p->pt_mean = 0.6;
    p->eta_max = 0.9;
    p->zv_sigma = 5.0;
    p->vdrift = 2.58;
    p->drift_len = 250.0;
    p->n_threads = 8;
}

synth_frame *synth_generate(const synth_params *p) {
    synth_frame *f = (synth_frame *)calloc(1, sizeof(synth_frame));
    int32_t nc = p->n_collisions;
    if (nc < 0) nc = 0;
    /* frame-level draws: collision time, vertex z, multiplicity */
    syn_rng fr = syn_stream(p->seed, 0);
    double *tc = (double *)malloc(sizeof(double) * (nc + 1));
    double *zv = (double *)malloc(sizeof(double) * (nc + 1));
    int64_t *first = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
    first[0] = 0;
    for (int32_t c = 0; c < nc; c++) {
        tc[c] = p->single_sector ? 0.0 : p->frame_us * syn_unif(&fr);
        zv[c] = p->zv_sigma * syn_normal(&fr);
        int64_t m;
        if (p->fixed_mult > 0) {
            m = p->fixed_mult;
        } else {
            double v;
            do { v = syn_exp(&fr, p->mult_mean); } while (v > p->mult_max);
            m = (int64_t)llround(v);
        }
        first[c + 1] = first[c] + m;
    }
    f->n_tracks = first[nc];
    f->tracks = (syn_track *)calloc((size_t)(f->n_tracks ? f->n_tracks : 1), sizeof(syn_track));
    for (int32_t c = 0; c < nc; c++)
        for (int64_t j = first[c]; j < first[c + 1]; j++) {
            f->tracks[j].zv = zv[c];
            f->tracks[j].tcoll_us = tc[c];
        }
    if (p->single_sector) {
        f->t_lo = -p->drift_len;
        f->t_hi = p->drift_len;
    } else {
        f->t_lo = 0.0;
        f->t_hi = p->vdrift * p->frame_us + p->drift_len;
    }

    syn_job jb;
    jb.p = p;
    jb.tracks = f->tracks;
    jb.first_track = first;
    jb.bufs = (syn_buf *)calloc((size_t)(nc ? nc : 1), sizeof(syn_buf));
    jb.n_coll = nc;
    jb.next = 0;
    pthread_mutex_init(&jb.mu, NULL);
    int nt = p->n_threads < 1 ? 1 : (p->n_threads > 64 ? 64 : p->n_threads);
    pthread_t th[64];
    for (int i = 0; i < nt; i++) pthread_create(&th[i], NULL, syn_worker, &jb);
    for (int i = 0; i < nt; i++) pthread_join(th[i], NULL);
    pthread_mutex_destroy(&jb.mu);

    /* merge in collision order */
    for (int32_t c = 0; c < nc; c++)
        for (int64_t i = 0; i < jb.bufs[c].n; i++) f->n[jb.bufs[c].v[i].sector]++;
    int64_t cur[SYN_NSECT];
    for (int s = 0; s < SYN_NSECT; s++) {
        int64_t n = f->n[s] ? f->n[s] : 1;
        f->row[s] = (uint8_t *)malloc((size_t)n);
        f->y[s] = (float *)malloc((size_t)n * 4);
        f->t[s] = (float *)malloc((size_t)n * 4);
        f->label[s] = (int32_t *)malloc((size_t)n * 4);
        cur[s] = 0;
    }
    for (int32_t c = 0; c < nc; c++) {
        for (int64_t i = 0; i < jb.bufs[c].n; i++) {
            syn_rec *r = &jb.bufs[c].v[i];
            int s = r->sector;
            int64_t k = cur[s]++;
            f->row[s][k] = r->row;
            f->y[s][k] = r->y;
            f->t[s][k] = r->t;
            f->label[s][k] = r->label;
        }
        free(jb.bufs[c].v);
    }
    free(jb.bufs);
    free(tc);
    free(zv);
    free(first);

    syn_noise_job nj;
    nj.p = p;
    nj.f = f;
    nj.next = p->single_sector ? SYN_NSECT - 1 : 0;
    pthread_mutex_init(&nj.mu, NULL);
    if (p->single_sector) {
        syn_noise_sector(p, f, 0);
    } else {
        for (int i = 0; i < nt; i++) pthread_create(&th[i], NULL, syn_noise_worker, &nj);
        for (int i = 0; i < nt; i++) pthread_join(th[i], NULL);
    }
    pthread_mutex_destroy(&nj.mu);
    return f;
}

int64_t synth_sector_count(const synth_frame *f, int32_t s) {
    return (s >= 0 && s < SYN_NSECT) ? f->n[s] : 0;
}

void synth_sector_copy(const synth_frame *f, int32_t s, uint8_t *row, float *y, float *t, int32_t *label) {
    if (s < 0 || s >= SYN_NSECT) return;
    int64_t n = f->n[s];
    if (row) memcpy(row, f->row[s], (size_t)n);
    if (y) memcpy(y, f->y[s], (size_t)n * 4);
    if (t) memcpy(t, f->t[s], (size_t)n * 4);
    if (label) memcpy(label, f->label[s], (size_t)n * 4);
}

int64_t synth_n_tracks(const synth_frame *f) { return f->n_tracks; }

/* Truth per track: q, pt, phi0, tgl, zv, tcoll_us, kappa, eta. */
void synth_tracks_copy(const synth_frame *f, double *out8) {
    for (int64_t j = 0; j < f->n_tracks; j++) {
        const syn_track *tr = &f->tracks[j];
        double *o = out8 + 8 * j;
        o[0] = tr->q; o[1] = tr->pt; o[2] = tr->phi0; o[3] = tr->tgl;
        o[4] = tr->zv; o[5] = tr->tcoll_us; o[6] = tr->kappa; o[7] = tr->eta;
    }
}

void synth_time_range(const synth_frame *f, double *lo, double *hi) {
    *lo = f->t_lo;
    *hi = f->t_hi;
}

void synth_free(synth_frame *f) {
    if (!f) return;
    for (int s = 0; s < SYN_NSECT; s++) {
        free(f->row[s]); free(f->y[s]); free(f->t[s]); free(f->label[s]);
    }
    free(f->tracks);
    free(f);
}

/*
 * Truth helix of one generated track at the row line X = x of a sector's
 * local frame (rising crossing, outgoing half turn). Fills
 * out[0..5] = Y, z, sin(local phi), arc length, time (cm, by the same rule as
 * the clusters; single_sector: t = z), dt/darc. Returns 0 when the helix does
 * not cross the line.
 */
int32_t synth_helix_at(const double *trk8, int32_t sector, double x, int32_t single_sector,
                       double vdrift, double drift_len, double *out) {
    syn_track tr;
    memset(&tr, 0, sizeof(tr));
    tr.q = trk8[0]; tr.pt = trk8[1]; tr.phi0 = trk8[2]; tr.tgl = trk8[3];
    tr.zv = trk8[4]; tr.tcoll_us = trk8[5]; tr.kappa = trk8[6];
    double al = syn_alpha(sector);
    double Y, arc;
    if (!syn_cross(&tr, al, x, &Y, &arc)) return 0;
    double z = tr.zv + tr.tgl * arc;
    double pl = tr.phi0 - al + tr.kappa * arc;
    out[0] = Y;
    out[1] = z;
    out[2] = sin(pl);
    out[3] = arc;
    if (single_sector) {
        out[4] = z;
        out[5] = tr.tgl;
    } else {
        out[4] = vdrift * tr.tcoll_us + (drift_len - fabs(z));
        out[5] = (sector < 18) ? -tr.tgl : tr.tgl;
    }
    return 1;
}
