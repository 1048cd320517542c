/*
 * Seeded synthetic initial configurations: random sequential insertion (RSA)
 * of equal hard disks into a square box with hard walls.
 *
 * This is an input generator only.  It holds none of the simulation method's
 * arithmetic: both the GPU library and the CPU oracle consume its output.
 *
 * Candidate centres are uniform in [r, L-r]^2 and a candidate is rejected when
 * it lies closer than 2r to any disk already placed.  Disks are numbered in the
 * order they were accepted.  Random numbers come from SplitMix64 (Steele, Lea
 * and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static uint64_t splitmix64_next(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static double unit53(uint64_t *s) { return (double)(splitmix64_next(s) >> 11) * 0x1.0p-53; }

/*
 * Places n disks of radius r in [0,L]^2.  Returns 0 on success, -1 on bad
 * arguments, -2 when max_attempts candidates were drawn before n were placed,
 * -3 on allocation failure.  xy_out holds 2n doubles (x0,y0,x1,y1,...).
 */
int rsa_disks(int n, double L, double r, uint64_t seed, long long max_attempts,
              double *xy_out, long long *attempts_out) {
    if (n < 0 || !(L > 2.0 * r) || !(r > 0.0) || xy_out == NULL) return -1;
    const double span = L - 2.0 * r;
    const double cell = 2.0 * r;
    long long nc = (long long)floor(L / cell);
    if (nc < 1) nc = 1;
    if (nc > 65536) nc = 65536;
    const double inv_cell = (double)nc / L;
    int *head = (int *)malloc(sizeof(int) * (size_t)(nc * nc));
    int *next = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!head || !next) {
        free(head);
        free(next);
        return -3;
    }
    for (long long c = 0; c < nc * nc; ++c) head[c] = -1;
    uint64_t state = seed ^ 0x5DEECE66DULL;
    const double min_d2 = 4.0 * r * r;
    long long attempts = 0;
    int placed = 0;
    while (placed < n) {
        if (attempts >= max_attempts) break;
        ++attempts;
        double x = r + span * unit53(&state);
        double y = r + span * unit53(&state);
        long long cx = (long long)(x * inv_cell), cy = (long long)(y * inv_cell);
        if (cx >= nc) cx = nc - 1;
        if (cy >= nc) cy = nc - 1;
        int ok = 1;
        for (long long gy = cy - 1; gy <= cy + 1 && ok; ++gy) {
            if (gy < 0 || gy >= nc) continue;
            for (long long gx = cx - 1; gx <= cx + 1 && ok; ++gx) {
                if (gx < 0 || gx >= nc) continue;
                for (int k = head[gy * nc + gx]; k >= 0; k = next[k]) {
                    double dx = x - xy_out[2 * k], dy = y - xy_out[2 * k + 1];
                    if (dx * dx + dy * dy < min_d2) {
                        ok = 0;
                        break;
                    }
                }
            }
        }
        if (!ok) continue;
        xy_out[2 * placed] = x;
        xy_out[2 * placed + 1] = y;
        next[placed] = head[cy * nc + cx];
        head[cy * nc + cx] = placed;
        ++placed;
    }
    free(head);
    free(next);
    if (attempts_out) *attempts_out = attempts;
    return placed == n ? 0 : -2;
}

/*
 * The same in a periodic box [0,L)^2: candidate centres are uniform in
 * [0,L)^2 and separations are taken from the nearest periodic image.  Same
 * return codes.
 */
int rsa_disks_periodic(int n, double L, double r, uint64_t seed, long long max_attempts,
                       double *xy_out, long long *attempts_out) {
    if (n < 0 || !(L > 2.0 * r) || !(r > 0.0) || xy_out == NULL) return -1;
    long long nc = (long long)floor(L / (2.0 * r));
    if (nc > 65536) nc = 65536;
    const int brute = nc < 3;   /* fewer than 3 cells a side: test every placed disk */
    if (nc < 1) nc = 1;
    const double inv_cell = (double)nc / L;
    int *head = (int *)malloc(sizeof(int) * (size_t)(nc * nc));
    int *next = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!head || !next) {
        free(head);
        free(next);
        return -3;
    }
    for (long long c = 0; c < nc * nc; ++c) head[c] = -1;
    uint64_t state = seed ^ 0x9A3D1C5B7ULL;
    const double min_d2 = 4.0 * r * r;
    long long attempts = 0;
    int placed = 0;
    while (placed < n) {
        if (attempts >= max_attempts) break;
        ++attempts;
        double x = L * unit53(&state);
        double y = L * unit53(&state);
        long long cx = (long long)(x * inv_cell), cy = (long long)(y * inv_cell);
        if (cx >= nc) cx = nc - 1;
        if (cy >= nc) cy = nc - 1;
        int ok = 1;
        if (brute) {
            for (int k = 0; k < placed && ok; ++k) {
                double dx = x - xy_out[2 * k], dy = y - xy_out[2 * k + 1];
                dx -= L * nearbyint(dx / L);
                dy -= L * nearbyint(dy / L);
                if (dx * dx + dy * dy < min_d2) ok = 0;
            }
        } else {
            for (long long gy = cy - 1; gy <= cy + 1 && ok; ++gy) {
                long long wy = (gy + nc) % nc;
                for (long long gx = cx - 1; gx <= cx + 1 && ok; ++gx) {
                    long long wx = (gx + nc) % nc;
                    for (int k = head[wy * nc + wx]; k >= 0; k = next[k]) {
                        double dx = x - xy_out[2 * k], dy = y - xy_out[2 * k + 1];
                        dx -= L * nearbyint(dx / L);
                        dy -= L * nearbyint(dy / L);
                        if (dx * dx + dy * dy < min_d2) {
                            ok = 0;
                            break;
                        }
                    }
                }
            }
        }
        if (!ok) continue;
        xy_out[2 * placed] = x;
        xy_out[2 * placed + 1] = y;
        next[placed] = head[cy * nc + cx];
        head[cy * nc + cx] = placed;
        ++placed;
    }
    free(head);
    free(next);
    if (attempts_out) *attempts_out = attempts;
    return placed == n ? 0 : -2;
}
