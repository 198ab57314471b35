/* The batching configuration's application (one instance;
 * sizes are set per instance) as C loop nests (parsed by paper_1806_01430_amd.cfront
 * into the same description as batch.json). */
#define N 64
#define I 17
#define J 17
#define K 33
#define SWEEPS 10
#define MODE 1

float A[N][N];
float B[N][N];
float C[N][N];          // ofl: output
float p[I][J][K];       // ofl: output setup=sin mode=MODE
float q[I][J][K];
double res[SWEEPS];     // ofl: output

/* random inputs: counter-based uniform streams 0 and 1 */
for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++) {
        A[i][j] = u01(0, i, j);
        B[i][j] = u01(1, i, j);
    }

/* C = A B */
for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++) {
        C[i][j] = 0.0f;
        for (int k = 0; k < N; k++)
            C[i][j] += A[i][k] * B[k][j];
    }

/* SWEEPS weighted-Jacobi sweeps of the 19-point neighbourhood */
for (int n = 0; n < SWEEPS; n++) {
    for (int i = 1; i < I - 1; i++)
        for (int j = 1; j < J - 1; j++)
            for (int k = 1; k < K - 1; k++) {
                float xm = (p[i - 1][j - 1][k] + p[i - 1][j + 1][k]) + (p[i - 1][j][k - 1] + p[i - 1][j][k + 1]);
                float x0 = (p[i][j - 1][k] + p[i][j + 1][k]) + (p[i][j][k - 1] + p[i][j][k + 1]);
                float xp = (p[i + 1][j - 1][k] + p[i + 1][j + 1][k]) + (p[i + 1][j][k - 1] + p[i + 1][j][k + 1]);
                float y0 = (p[i][j - 1][k - 1] + p[i][j - 1][k + 1]) + (p[i][j + 1][k - 1] + p[i][j + 1][k + 1]);
                float faces = (p[i - 1][j][k] + p[i + 1][j][k]) + x0;
                float edges = (xm + xp) + y0;
                float r = (0.25f * p[i][j][k] + 0.0625f * faces) + 0.03125f * edges;
                q[i][j][k] = r;
                double d = (double)r - (double)p[i][j][k];
                res[n] += d * d;
            }
    for (int i = 1; i < I - 1; i++)
        for (int j = 1; j < J - 1; j++)
            for (int k = 1; k < K - 1; k++)
                p[i][j][k] = q[i][j][k];
}
