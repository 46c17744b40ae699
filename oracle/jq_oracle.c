/*
 * Plain CPU oracle for state-vector gate application (De Raedt et al.,
 * "Massively parallel quantum computer simulator, eleven years later").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and is
 * loaded by the tests, by the smoke check and by the CPU-baseline leg of the
 * benchmark.  The product library never links, loads or calls it, and it
 * shares no source with the GPU path.
 *
 * Everything here is the slow, obvious definition: one amplitude group at a
 * time, FP64, single thread, built with -O2 -ffp-contract=off so every
 * multiply and add rounds on its own.
 *
 * State layout (Sec. 2, Eq. STAT2): 2^N complex amplitudes, interleaved
 * (re, im) doubles; qubit j is bit j of the basis index, qubit 0 the least
 * significant bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/*
 * Projection of qubit q onto |v> with renormalisation (App. A, CLEAR for
 * v = 0 and SET for v = 1: |v><v| on qubit q): p is the sum of |a_i|^2 over
 * the indices whose bit q equals v; those amplitudes are divided by sqrt(p)
 * and all others set to zero.  Returns p.  If p == 0 the projected state
 * has zero amplitude (the paper's instructions fail then) and the state is
 * left unchanged.
 */
double oq_project(double *psi, int n, int q, int v)
{
    const uint64_t dim = 1ull << n, b = 1ull << q;
    double p = 0.0;
    for (uint64_t i = 0; i < dim; i++)
        if (((i & b) != 0) == (v != 0)) p = p + (psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1]);
    if (p == 0.0) return 0.0;
    const double f = 1.0 / sqrt(p);
    for (uint64_t i = 0; i < dim; i++) {
        if (((i & b) != 0) == (v != 0)) {
            psi[2 * i] = psi[2 * i] * f;
            psi[2 * i + 1] = psi[2 * i + 1] * f;
        } else {
            psi[2 * i] = 0.0;
            psi[2 * i + 1] = 0.0;
        }
    }
    return p;
}

/*
 * Projective measurement of qubit q (App. A, M): p0 and p1 are the
 * probabilities of outcomes 0 and 1 (sums of |a_i|^2 over bit q = 0, 1);
 * the outcome is 1 when u >= p0 / (p0 + p1) for the caller's draw u in
 * [0, 1), else 0, and the state is projected onto it as by oq_project.
 * *p1_out receives p1 / (p0 + p1).  Returns the outcome, or -1 if the state
 * is zero.
 */
int oq_measure(double *psi, int n, int q, double u, double *p1_out)
{
    const uint64_t dim = 1ull << n, b = 1ull << q;
    double p0 = 0.0, p1 = 0.0;
    for (uint64_t i = 0; i < dim; i++) {
        double m = psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1];
        if (i & b) p1 = p1 + m; else p0 = p0 + m;
    }
    if (p0 + p1 == 0.0) return -1;
    *p1_out = p1 / (p0 + p1);
    const int outcome = u >= p0 / (p0 + p1) ? 1 : 0;
    oq_project(psi, n, q, outcome);
    return outcome;
}

/*
 * Sampling of basis states (App. A, GENERATE EVENTS): with the cumulative
 * sums C_i = p_0 + ... + p_i of p_i = |a_i|^2 (accumulated in index order)
 * and the caller's draws u_k in [0, 1), event k is the least i with
 * C_i > u_k * C_(2^N - 1).  Returns 0, or -1 for a zero state.
 */
int oq_sample(const double *psi, int n, const double *u, int count, uint64_t *out)
{
    const uint64_t dim = 1ull << n;
    double *cdf = (double *)malloc(dim * sizeof(double));
    if (!cdf) return -1;
    double c = 0.0;
    for (uint64_t i = 0; i < dim; i++) {
        c = c + (psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1]);
        cdf[i] = c;
    }
    if (c == 0.0) { free(cdf); return -1; }
    for (int k = 0; k < count; k++) {
        const double t = u[k] * c;
        uint64_t lo = 0, hi = dim - 1;  /* cdf[hi] = c > t */
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > t) hi = mid; else lo = mid + 1;
        }
        out[k] = lo;
    }
    free(cdf);
    return 0;
}

/*
 * Apply a 2^k x 2^k matrix to the target qubits targets[0..k-1] on the
 * subspace where every control qubit is 1 (Sec. 2, Eq. NUM2 for k = 1; the
 * groups of four and eight amplitudes for k = 2, 3).  Row/column index of
 * the matrix: targets[0] is the most significant bit, as in the basis
 * |control,target> of the CNOT definition (App. A).  The matrix is row-major
 * with interleaved (re, im) entries.
 *
 * Returns 0, or -1 on invalid arguments (the state is then untouched).
 */
int oq_apply(double *psi, int n, const int *targets, int k,
             const int *controls, int nc, const double *m)
{
    if (n < 1 || n > 40 || k < 1 || k > 3 || nc < 0 || nc > 8) return -1;
    uint64_t tmask = 0, cmask = 0;
    for (int s = 0; s < k; s++) {
        if (targets[s] < 0 || targets[s] >= n) return -1;
        if (tmask & (1ull << targets[s])) return -1;
        tmask |= 1ull << targets[s];
    }
    for (int s = 0; s < nc; s++) {
        if (controls[s] < 0 || controls[s] >= n) return -1;
        uint64_t b = 1ull << controls[s];
        if ((tmask | cmask) & b) return -1;
        cmask |= b;
    }
    const uint64_t dim = 1ull << n;
    const int K = 1 << k;
    uint64_t idx[8];
    double in_re[8], in_im[8];
    for (uint64_t i = 0; i < dim; i++) {
        if (i & tmask) continue;              /* i is the group's base */
        if ((i & cmask) != cmask) continue;   /* controls not all 1 */
        for (int a = 0; a < K; a++) {
            uint64_t j = i;
            for (int s = 0; s < k; s++)
                if ((a >> (k - 1 - s)) & 1) j |= 1ull << targets[s];
            idx[a] = j;
            in_re[a] = psi[2 * j];
            in_im[a] = psi[2 * j + 1];
        }
        for (int r = 0; r < K; r++) {
            double sr = 0.0, si = 0.0;
            for (int c = 0; c < K; c++) {
                double mr = m[2 * (r * K + c)], mi = m[2 * (r * K + c) + 1];
                sr = sr + (mr * in_re[c] - mi * in_im[c]);
                si = si + (mr * in_im[c] + mi * in_re[c]);
            }
            psi[2 * idx[r]] = sr;
            psi[2 * idx[r] + 1] = si;
        }
    }
    return 0;
}

/* Squared norm, the left side of Eq. STAT1, summed in index order. */
double oq_norm2(const double *psi, int n)
{
    const uint64_t dim = 1ull << n;
    double s = 0.0;
    for (uint64_t i = 0; i < dim; i++)
        s = s + (psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1]);
    return s;
}

/*
 * Marginal distribution over qubits[0..nq-1] (Sec. 2: the probability of
 * outcome 0/1 on qubit j is the sum of |a|^2 over indices with that bit).
 * out has 2^nq entries; bit m of the output index is the value of
 * qubits[m].  Summed in index order.
 */
int oq_probabilities(const double *psi, int n, const int *qubits, int nq,
                     double *out)
{
    if (nq < 0 || nq > n || nq > 30) return -1;
    for (int m = 0; m < nq; m++)
        if (qubits[m] < 0 || qubits[m] >= n) return -1;
    const uint64_t nb = 1ull << nq;
    for (uint64_t b = 0; b < nb; b++) out[b] = 0.0;
    const uint64_t dim = 1ull << n;
    for (uint64_t i = 0; i < dim; i++) {
        uint64_t b = 0;
        for (int m = 0; m < nq; m++) b |= ((i >> qubits[m]) & 1ull) << m;
        out[b] = out[b] + (psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1]);
    }
    return 0;
}

/*
 * Expectation values of App. A, BEGIN MEASUREMENT:
 * <Q_alpha(n)> = <Psi|(1 - sigma^alpha_n)|Psi>/2 for alpha = x, y, z.
 * Computed from the definition: sigma^x flips bit n, sigma^y flips it with
 * a factor +i (bit 0 -> 1) or -i (bit 1 -> 0) on the new amplitude, sigma^z
 * multiplies by +1/-1.  Divided by <Psi|Psi> so an unnormalised state still
 * gives the expectation of the normalised one.
 */
void oq_expect_q(const double *psi, int n, double *qx, double *qy, double *qz)
{
    const uint64_t dim = 1ull << n;
    double nrm = oq_norm2(psi, n);
    for (int q = 0; q < n; q++) {
        const uint64_t b = 1ull << q;
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (uint64_t i = 0; i < dim; i++) {
            uint64_t j = i ^ b;
            double ar = psi[2 * i], ai = psi[2 * i + 1];
            double cr = psi[2 * j], ci = psi[2 * j + 1];
            /* (sigma^x psi)_i = psi_j ; contribution conj(psi_i) psi_j */
            sx = sx + (ar * cr + ai * ci);
            /* (sigma^y psi)_i = -i psi_j if bit q of i is 0, +i psi_j if 1 */
            double yr, yi;
            if (i & b) { yr = -ci; yi = cr; } else { yr = ci; yi = -cr; }
            sy = sy + (ar * yr + ai * yi);
            double p = ar * ar + ai * ai;
            sz = sz + ((i & b) ? -p : p);
        }
        qx[q] = (1.0 - sx / nrm) / 2.0;
        qy[q] = (1.0 - sy / nrm) / 2.0;
        qz[q] = (1.0 - sz / nrm) / 2.0;
    }
}

/* ------------------------------------------------------------------------
 * The adaptive two-byte polar encoding of Sec. 4.1.
 *
 * b1 in [-128, 128) encodes the angle theta = pi*b1/128.  b0 encodes the
 * modulus: -128 is r = 0, 127 is r = 1, and every other code c gives
 * r = (c+127)(r1-r0)/253 + r0, where r0, r1 are the smallest and largest
 * |z| with 0 < |z| < 1 over the state.  Codes are stored as two planes,
 * b0[2^N] then b1[2^N].
 *
 * Readings taken where the text is silent:
 *  - rounding is round-half-even (rint); b0 is clamped to [-127, 126];
 *  - a modulus counts as zero only when it is exactly 0.0 and as one when
 *    it is >= 1 - ONE_TOL, so that a basis state that picked up a phase
 *    (|z| = 1 - 1ulp) keeps its exact code;
 *  - a zero amplitude has b1 = 0; atan2's +pi maps to code -128;
 *  - r1 == r0 encodes every in-range modulus as -127;
 *  - the range (r0, r1) is recomputed over the whole state after every
 *    gate; a permutation gate or a diagonal gate whose entries all have
 *    modulus 1 keeps it; if no modulus lies strictly between zero and one
 *    the previous range is kept.
 * ---------------------------------------------------------------------- */
#define ONE_TOL 1e-12

static void decode1(int8_t c0, int8_t c1, double r0, double r1,
                    double *re, double *im)
{
    if (c0 == -128) { *re = 0.0; *im = 0.0; return; }
    double r;
    if (c0 == 127) r = 1.0;
    else r = ((double)((int)c0 + 127) * (r1 - r0)) / 253.0 + r0;
    double th = (M_PI * (double)c1) / 128.0;
    *re = r * cos(th);
    *im = r * sin(th);
}

static void encode1(double re, double im, double r0, double r1,
                    int8_t *c0, int8_t *c1)
{
    double a = sqrt(re * re + im * im);
    if (a == 0.0) { *c0 = -128; *c1 = 0; return; }
    if (a >= 1.0 - ONE_TOL) {
        *c0 = 127;
    } else if (r1 == r0) {
        *c0 = -127;
    } else {
        double q = rint((253.0 * (a - r0)) / (r1 - r0));
        long v = -127 + (long)q;
        if (v < -127) v = -127;
        if (v > 126) v = 126;
        *c0 = (int8_t)v;
    }
    long t = (long)rint((128.0 * atan2(im, re)) / M_PI);
    if (t >= 128) t -= 256;
    if (t < -128) t += 256;
    *c1 = (int8_t)t;
}

void oq_compact_decode(const int8_t *b0, const int8_t *b1, uint64_t count,
                       double r0, double r1, double *psi)
{
    for (uint64_t i = 0; i < count; i++)
        decode1(b0[i], b1[i], r0, r1, &psi[2 * i], &psi[2 * i + 1]);
}

void oq_compact_encode(const double *psi, uint64_t count, double r0,
                       double r1, int8_t *b0, int8_t *b1)
{
    for (uint64_t i = 0; i < count; i++)
        encode1(psi[2 * i], psi[2 * i + 1], r0, r1, &b0[i], &b1[i]);
}

/* min and max of |z| over 0 < |z| < 1 (the "one" tolerance as in encode1).
 * Returns 1 and writes r0, r1 if such an element exists, else returns 0. */
int oq_compact_range(const double *psi, uint64_t count, double *r0, double *r1)
{
    int found = 0;
    double lo = 0.0, hi = 0.0;
    for (uint64_t i = 0; i < count; i++) {
        double a = sqrt(psi[2 * i] * psi[2 * i] + psi[2 * i + 1] * psi[2 * i + 1]);
        if (a == 0.0 || a >= 1.0 - ONE_TOL) continue;
        if (!found) { lo = a; hi = a; found = 1; }
        else { if (a < lo) lo = a; if (a > hi) hi = a; }
    }
    if (found) { *r0 = lo; *r1 = hi; }
    return found;
}

/* Is the 2^k x 2^k matrix a permutation (entries exactly 0 or 1, one 1 per
 * row and column)?  Is it diagonal with every entry of modulus 1? */
static int is_permutation(const double *m, int K)
{
    for (int r = 0; r < K; r++) {
        int ones = 0;
        for (int c = 0; c < K; c++) {
            double re = m[2 * (r * K + c)], im = m[2 * (r * K + c) + 1];
            if (im != 0.0) return 0;
            if (re == 1.0) ones++;
            else if (re != 0.0) return 0;
        }
        if (ones != 1) return 0;
    }
    for (int c = 0; c < K; c++) {
        int ones = 0;
        for (int r = 0; r < K; r++) if (m[2 * (r * K + c)] == 1.0) ones++;
        if (ones != 1) return 0;
    }
    return 1;
}

static int is_unimodular_diagonal(const double *m, int K)
{
    for (int r = 0; r < K; r++)
        for (int c = 0; c < K; c++) {
            double re = m[2 * (r * K + c)], im = m[2 * (r * K + c) + 1];
            if (r != c) { if (re != 0.0 || im != 0.0) return 0; }
            else if (fabs(sqrt(re * re + im * im) - 1.0) > ONE_TOL) return 0;
        }
    return 1;
}

/* One gate record for the whole-circuit entry points below. */
typedef struct {
    int k;            /* number of targets, 1..3 */
    int nc;           /* number of controls, 0..8 */
    int targets[3];   /* targets[0] is the MSB of the matrix index */
    int controls[8];
    double m[128];    /* 2^k x 2^k row-major, interleaved (re, im) */
} oq_gate;

/* Apply gates[0..count-1] in order (Sec. 2: a circuit is a sequence of
 * unitary operations on the state). */
int oq_run(double *psi, int n, const oq_gate *gates, int count)
{
    for (int g = 0; g < count; g++) {
        int rc = oq_apply(psi, n, gates[g].targets, gates[g].k,
                          gates[g].controls, gates[g].nc, gates[g].m);
        if (rc) return rc;
    }
    return 0;
}

/*
 * A run of gates in the encoded flavour (Sec. 4.1): decode every amplitude
 * with the current (r0, r1), apply the gates in FP64 exactly as oq_apply
 * does, choose the new range, encode every amplitude.  With count == 1 this
 * is the paper's per-gate procedure; a longer run quantises once per run.
 * The range is kept when every gate of the run is a permutation or a
 * diagonal of modulus-one entries, and when no modulus lies strictly
 * between zero and one.  rng[0..1] holds (r0, r1) on entry and the new
 * range on exit.  scratch must hold 2^(n+1) doubles.
 */
int oq_compact_run(int8_t *b0, int8_t *b1, int n, double *rng,
                   const oq_gate *gates, int count, double *scratch)
{
    const uint64_t dim = 1ull << n;
    oq_compact_decode(b0, b1, dim, rng[0], rng[1], scratch);
    int keep = 1;
    for (int g = 0; g < count; g++) {
        int rc = oq_apply(scratch, n, gates[g].targets, gates[g].k,
                          gates[g].controls, gates[g].nc, gates[g].m);
        if (rc) return rc;
        int K = 1 << gates[g].k;
        if (!(is_permutation(gates[g].m, K) || is_unimodular_diagonal(gates[g].m, K)))
            keep = 0;
    }
    if (!keep) {
        double lo, hi;
        if (oq_compact_range(scratch, dim, &lo, &hi)) { rng[0] = lo; rng[1] = hi; }
    }
    oq_compact_encode(scratch, dim, rng[0], rng[1], b0, b1);
    return 0;
}
