/* Plain C CIC deposit for the oracle (TEST INFRASTRUCTURE ONLY: nothing in the
 * product path may link, load or call it).  It computes the same definition as
 * oracle/cwthf.py's deposit (Sec. 2 step 2, Eq. (1)) for boxes too large for
 * NumPy's add.at, one particle at a time in input order, with no blocking and
 * no reordering.  It shares no code with the GPU library.
 *
 * Per axis the position x becomes q = floor(fl(x * s)) mod n 2^B, with
 * s = n 2^B / L rounded once to the position type and one correctly rounded
 * multiply in that type (this file is compiled without FMA contraction and
 * without fast-math); the cell is q >> B, the fraction f = q & (2^B - 1), and
 * the lower and upper nodes weigh 2^B - f and f.  Each of the eight corners
 * (periodic) gets the product of its three weights, added exactly in int64;
 * a cell sum above 2^63 - 1 is reported (return 2), a non-finite or
 * out-of-range position too (return 1).  rho is [n][n][n] (z, y, x), zeroed
 * by the caller.  Only corners on the z planes [z0, z1) are added, so that
 * disjoint plane ranges can be filled by independent calls (each cell's sum is
 * the same whichever call makes it). */
#include <math.h>
#include <stdint.h>

static int axis_q(double t, int64_t m, int64_t *q) {
    if (!(t == t) || fabs(t) >= 4611686018427387904.0) return 1; /* NaN, inf or |t| >= 2^62 */
    int64_t v = (int64_t)floor(t) % m;
    if (v < 0) v += m;
    *q = v;
    return 0;
}

/* Whether either z node of a particle (cell and cell + 1, periodic) lies in
 * [z0, z1); particles that touch no plane of the range add nothing there (their
 * x and y coordinates are then not examined by this call). */
static int touches(int64_t qz, int n, int frac_bits, int64_t z0, int64_t z1) {
    const int64_t c0 = qz >> frac_bits, c1 = (c0 + 1) % n;
    return (c0 >= z0 && c0 < z1) || (c1 >= z0 && c1 < z1);
}

static int add_particle(const int64_t q[3], int n, int frac_bits, int64_t z0, int64_t z1, int64_t *rho) {
    const int64_t one = (int64_t)1 << frac_bits;
    int64_t cell[3], w[3][2];
    for (int a = 0; a < 3; ++a) {
        const int64_t f = q[a] & (one - 1);
        cell[a] = q[a] >> frac_bits;
        w[a][0] = one - f;
        w[a][1] = f;
    }
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                const int64_t iz = (cell[2] + cz) % n, iy = (cell[1] + cy) % n, ix = (cell[0] + cx) % n;
                if (iz < z0 || iz >= z1) continue;
                const int64_t wt = w[2][cz] * w[1][cy] * w[0][cx];
                int64_t *r = &rho[(iz * n + iy) * n + ix];
                if (__builtin_add_overflow(*r, wt, r)) return 2;
            }
    return 0;
}

int oracle_cic_deposit_f32(const float *pos, int64_t np, double box_len, int n, int frac_bits, int64_t z0,
                           int64_t z1, int64_t *rho) {
    const int64_t m = (int64_t)n << frac_bits;
    const float s = (float)((double)n * (double)((int64_t)1 << frac_bits) / box_len);
    for (int64_t p = 0; p < np; ++p) {
        int64_t q[3];
        if (axis_q((double)(pos[3 * p + 2] * s), m, &q[2])) return 1;
        if (!touches(q[2], n, frac_bits, z0, z1)) continue;
        for (int a = 0; a < 2; ++a) {
            const float t = pos[3 * p + a] * s;
            if (axis_q((double)t, m, &q[a])) return 1;
        }
        const int e = add_particle(q, n, frac_bits, z0, z1, rho);
        if (e) return e;
    }
    return 0;
}

int oracle_cic_deposit_f64(const double *pos, int64_t np, double box_len, int n, int frac_bits, int64_t z0,
                           int64_t z1, int64_t *rho) {
    const int64_t m = (int64_t)n << frac_bits;
    const double s = (double)n * (double)((int64_t)1 << frac_bits) / box_len;
    for (int64_t p = 0; p < np; ++p) {
        int64_t q[3];
        if (axis_q(pos[3 * p + 2] * s, m, &q[2])) return 1;
        if (!touches(q[2], n, frac_bits, z0, z1)) continue;
        for (int a = 0; a < 2; ++a) {
            const double t = pos[3 * p + a] * s;
            if (axis_q(t, m, &q[a])) return 1;
        }
        const int e = add_particle(q, n, frac_bits, z0, z1, rho);
        if (e) return e;
    }
    return 0;
}
