/* An application not written for offloading (Sec. 3.3: general programs).
 * Besides loops the library implements (a product, a transpose, the
 * iterated 19-point sweep and its copy, a sum of squares) it has loops that
 * no library operation matches -- index arithmetic, an update of part of an
 * array, double-precision arithmetic, a branch -- one that calls a math
 * routine and one that leaves early.  Those stay on the CPU, compiled from
 * their own text; the others each get a gene bit. */
#define N 200
#define H 72
#define I 21
#define J 19
#define K 67
#define SWEEPS 4

float A[N][N];          // ofl: output
float B[N][N];
float C[N][N];          // ofl: output
float E[N][N];          // ofl: output
double G[N][N];         // ofl: output
double T[N][N];         // ofl: output
float F[N][N];          // ofl: output
float r[N];             // ofl: output
double s[1];            // ofl: output
float p[I][J][K];       // ofl: output setup=sin mode=1
float q[I][J][K];
double res[SWEEPS];     // ofl: output

/* inputs from the element indices */
for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++) {
        A[i][j] = (float)((i * 37 + j * 11) % 101) * 0.01f + 0.05f;
        B[i][j] = (float)((i * 13 + j * 29) % 97) * 0.01f;
    }

/* C = A B */
for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++) {
        C[i][j] = 0.0f;
        for (int k = 0; k < N; k++)
            C[i][j] += A[i][k] * B[k][j];
    }

/* the first H rows only */
for (int i = 0; i < H; i++)
    for (int j = 0; j < N; j++)
        C[i][j] = C[i][j] + 0.5f * A[i][j];

/* a math routine */
for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++)
        E[i][j] = sqrtf(C[i][j]) + 1.0f;

/* double arithmetic */
for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++)
        G[i][j] = 0.1 * E[i][j] + (double)C[i][j];

/* a copy into a transposed double array: no library operation */
for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++)
        T[j][i] = G[i][j];

/* leaves at the first large diagonal value */
for (int i = 0; i < N; i++) {
    if (A[i][i] > 0.95f)
        break;
    r[i] = 2.0f * A[i][i] + 1.0f;
}

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
                float v = (0.25f * p[i][j][k] + 0.0625f * faces) + 0.03125f * edges;
                q[i][j][k] = v;
                double d = (double)v - (double)p[i][j][k];
                res[n] += d * d;
            }
    for (int i = 1; i < I - 1; i++)
        for (int j = 1; j < J - 1; j++)
            for (int k = 1; k < K - 1; k++)
                p[i][j][k] = q[i][j][k];
}

/* a branch in the body */
for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++) {
        float x = C[i][j] - 8.0f * E[i][j];
        if (x < 0.0f)
            x = -x;
        F[i][j] = x;
    }

/* the transpose of F into B */
for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++)
        B[j][i] = F[i][j];

for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++) {
        double u = (double)B[i][j];
        s[0] += u * u;
    }
