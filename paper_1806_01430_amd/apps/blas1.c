/* Level-1 BLAS library calls as function blocks (one gene bit each), beside
 * a loop nest of the same operation: saxpy, scopy and sscal on whole float
 * arrays become the nests of their loop forms. */
#define N 64
#define M 96

float X[N][M];
float Y[N][M];          // ofl: output
float Z[N][M];          // ofl: output

/* random inputs: counter-based uniform streams 0 and 1 */
for (int i = 0; i < N; i++)
    for (int j = 0; j < M; j++) {
        X[i][j] = u01(0, i, j);
        Y[i][j] = u01(1, i, j);
    }

saxpy(0.1, X, Y);       /* Y = Y + 0.1 X (alpha converted to float) */
scopy(Y, Z);            /* Z = Y */
sscal(-2.5f, Z);        /* Z = -2.5 Z */

/* the loop form of an axpy */
for (int i = 0; i < N; i++)
    for (int j = 0; j < M; j++)
        Z[i][j] = Z[i][j] + 0.5f * X[i][j];
