/* The spectral application as C (parsed by paper_1806_01430_amd.cfront into
 * the same description as spectral.json): R rows of n = M/2 complex samples,
 * real and imaginary parts interleaved. */
#define R 4096
#define M 2048

float X[R][M];          // ofl: output
double s[1];            // ofl: output

for (int i = 0; i < R; i++)
    for (int j = 0; j < M; j++)
        X[i][j] = u01(0, i, j);

/* library call: the forward DFT of every row */
fft_rows(X);

/* total energy of the spectra (n times the samples' energy) */
for (int i = 0; i < R; i++)
    for (int j = 0; j < M; j++) {
        double v = (double)X[i][j];
        s[0] += v * v;
    }

for (int i = 0; i < R; i++)
    for (int j = 0; j < M; j++)
        X[i][j] = 0.0009765625f * X[i][j];
