/* Host driver of the C oracle for sanitizer builds (AddressSanitizer,
 * UndefinedBehaviorSanitizer): every exported routine on a mesh read from
 * two raw files, with the hierarchy cast checked against brute force.
 * Usage: oracle_main VERTS.f32 N_VERTS TRIS.i32 N_TRIS.  Exit 0 on success. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_splitmix64(uint64_t seed, uint64_t c0, int64_t n, uint64_t *out);
void orc_fibonacci_dirs(int32_t n, float *out);
void orc_axes6(float *out);
void orc_frame(const float *n, float *t, float *b);
void orc_ray_dirs(const float *nrm, int64_t S, const float *dirs, int32_t N, int32_t kind, float *out);
void orc_mesh_info(const float *V, int64_t nv, double *bbox, double *diag, float *eps, float offset_frac);
int orc_area_weights(const float *V, const int32_t *T, int64_t nt, uint64_t *w, int32_t *k_out);
int orc_sample_area(const float *V, int64_t nv, const int32_t *T, int64_t nt, int64_t n, uint64_t seed,
                    float offset_frac, float *P, float *Nrm, float *O, int32_t *tri);
int64_t orc_sample_centroid(const float *V, int64_t nv, const int32_t *T, int64_t nt, float offset_frac, float *P,
                            float *Nrm, float *O, int32_t *tri);
int orc_cast(const float *V, int64_t nv, const int32_t *T, int64_t nt, const float *O, const float *Nrm, int64_t s0,
             int64_t s1, const float *dirs, int32_t N, int32_t kind, uint32_t *bits, uint32_t *grazing, uint32_t *info,
             int32_t nthreads);
int orc_cast_rays(const float *V, const int32_t *T, int64_t nt, const float *O, const float *D, int64_t nr, uint8_t *out,
                  int32_t nthreads);
void *orc_bvh_build(const float *V, int64_t nv, const int32_t *T, int64_t nt, double pad);
void orc_bvh_free(void *p);
void orc_bvh_shape(const void *p, int64_t *out);
int orc_bvh_cast(const void *ph, const float *O, const float *Nrm, int64_t s0, int64_t s1, const float *dirs, int32_t N,
                 int32_t kind, uint32_t *bits, uint32_t *grazing, uint32_t *info, uint64_t *work, int32_t nthreads);
int orc_cast_tool(const float *V, const int32_t *T, int64_t nt, const float *Pt, const float *Nrm, int64_t s0,
                  int64_t s1, const float *dirs, int32_t N, int32_t kind, double r, double tol, double band,
                  uint32_t *bits, uint32_t *amb, int32_t nthreads);
int orc_cast_tool_holder(const float *V, const int32_t *T, int64_t nt, const float *Pt, const float *Nrm, int64_t s0,
                         int64_t s1, const float *dirs, int32_t N, int32_t kind, double r, double len, double R,
                         double tol, double band, uint32_t *bits, uint32_t *amb, int32_t nthreads);
int orc_decide_one(const double *v9, const double *o, const double *d, int32_t *info);
void orc_dirstats(const float *Nrm, int64_t S, const float *dirs, int32_t N, const uint32_t *bits, double *mean,
                  double *absmean, int8_t *axis, double *conc, uint8_t *tie, uint64_t *hist);

static void *rd(const char *path, size_t bytes) {
    FILE *f = fopen(path, "rb");
    if (!f) exit(2);
    void *p = malloc(bytes);
    if (fread(p, 1, bytes, f) != bytes) exit(3);
    fclose(f);
    return p;
}

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                              \
        }                                                          \
    } while (0)

int main(int argc, char **argv) {
    if (argc != 5) return 2;
    const int64_t nv = atoll(argv[2]), nt = atoll(argv[4]);
    float *V = (float *)rd(argv[1], sizeof(float) * 3 * nv);
    int32_t *T = (int32_t *)rd(argv[3], sizeof(int32_t) * 3 * nt);
    uint64_t sm[4];
    orc_splitmix64(7, 0, 4, sm);
    const int32_t N = 96, W = (N + 31) / 32;
    float *dirs = malloc(sizeof(float) * 3 * N), ax[18];
    orc_fibonacci_dirs(N, dirs);
    orc_axes6(ax);
    double bbox[6], diag;
    float eps;
    orc_mesh_info(V, nv, bbox, &diag, &eps, 1e-4f);
    uint64_t *w = malloc(sizeof(uint64_t) * nt);
    int32_t k;
    CHECK(orc_area_weights(V, T, nt, w, &k) == 0);
    const int64_t S = 120;
    float *P = malloc(sizeof(float) * 3 * nt), *Nn = malloc(sizeof(float) * 3 * nt), *O = malloc(sizeof(float) * 3 * nt);
    int32_t *tri = malloc(sizeof(int32_t) * nt);
    CHECK(orc_sample_centroid(V, nv, T, nt, 1e-4f, P, Nn, O, tri) > 0);
    CHECK(orc_sample_area(V, nv, T, nt, S, 5, 1e-4f, P, Nn, O, tri) == 0);
    float t3[3], b3[3];
    orc_frame(Nn, t3, b3);
    float *rays = malloc(sizeof(float) * 3 * 4 * N);
    orc_ray_dirs(Nn, 4, dirs, N, 0, rays);
    uint32_t *bb = calloc(S * W, 4), *bg = calloc(S * W, 4), *bi = calloc(S * W, 4);
    uint32_t *hb = calloc(S * W, 4), *hg = calloc(S * W, 4), *hi = calloc(S * W, 4);
    CHECK(orc_cast(V, nv, T, nt, O, Nn, 0, S, dirs, N, 0, bb, bg, bi, 2) == 0);
    void *h = orc_bvh_build(V, nv, T, nt, 1e-4 * diag);
    CHECK(h != NULL);
    int64_t shape[2];
    orc_bvh_shape(h, shape);
    uint64_t work[2] = {0, 0};
    CHECK(orc_bvh_cast(h, O, Nn, 0, S, dirs, N, 0, hb, hg, hi, work, 2) == 0);
    for (int64_t q = 0; q < S * W; ++q) CHECK(((bb[q] ^ hb[q]) & ~bg[q]) == 0 && (hg[q] & ~bg[q]) == 0);
    uint32_t a6[120], g6[120], i6[120], h6[120], hg6[120], hi6[120];
    CHECK(orc_cast(V, nv, T, nt, O, Nn, 0, S, ax, 6, 1, a6, g6, i6, 2) == 0);
    CHECK(orc_bvh_cast(h, O, Nn, 0, S, ax, 6, 1, h6, hg6, hi6, NULL, 2) == 0);
    for (int64_t q = 0; q < S; ++q) CHECK(((a6[q] ^ h6[q]) & ~g6[q]) == 0);
    orc_bvh_free(h);
    uint8_t verdict[16];
    CHECK(orc_cast_rays(V, T, nt, O, rays, 16, verdict, 2) == 0);
    uint32_t tb[20 * 3], ta[20 * 3];
    CHECK(orc_cast_tool(V, T, nt, P, Nn, 0, 20, dirs, N, 0, 1.5, 1e-4 * diag, 1e-9 * diag, tb, ta, 2) == 0);
    CHECK(orc_cast_tool_holder(V, T, nt, P, Nn, 0, 20, dirs, N, 0, 1.5, 8.0, 4.0, 1e-4 * diag, 1e-9 * diag, tb, ta, 2) == 0);
    double v9[9], o[3] = {0, 0, 1}, d[3] = {0, 0, -1};
    for (int q = 0; q < 9; ++q) v9[q] = V[3 * T[q / 3] + q % 3];
    int32_t info;
    orc_decide_one(v9, o, d, &info);
    double *mean = malloc(sizeof(double) * 3 * S), *am = malloc(sizeof(double) * 3 * S), *conc = malloc(sizeof(double) * S);
    int8_t *axis = malloc(S);
    uint8_t *tie = malloc(S);
    uint64_t *hist = malloc(sizeof(uint64_t) * 8192);
    orc_dirstats(Nn, S, dirs, N, hb, mean, am, axis, conc, tie, hist);
    free(V); free(T); free(dirs); free(w); free(P); free(Nn); free(O); free(tri); free(rays);
    free(bb); free(bg); free(bi); free(hb); free(hg); free(hi);
    free(mean); free(am); free(conc); free(axis); free(tie); free(hist);
    printf("oracle ok: %lld nodes, depth %lld\n", (long long)shape[0], (long long)shape[1]);
    return 0;
}
