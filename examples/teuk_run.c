/*
 * teuk_run -- evolve one m-mode of the Teukolsky equation through the C ABI
 * of libteuk, with device buffers from the HIP runtime and no Python.
 *
 *   teuk_run IN OUT n_rstar n_theta rstar_min rstar_max a M m s dt r0 amp rstar_obs n_steps [prec]
 *
 * IN holds the initial Phi then Pi, each [n_theta][n_rstar] complex128
 * (interleaved re, im; r* contiguous).  The run takes n_steps Lax-Wendroff
 * steps (Eqs. 13-14) with the circular-orbit source of teuk_set_source
 * (amp = 0: none) and records the waveform at rstar_obs (Sec. 2.2).  OUT
 * receives the final Phi and Pi and then the waveform rows 0..n_steps, each
 * n_theta complex128.  prec is 64 (default) or 32; with 32 the state is
 * converted to complex64 on the host before the upload and back after.
 * Exit status 0 on success, 1 on a usage or I/O error, 2 on a library or
 * HIP error (the message goes to stderr).
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "teuk.h"

static int fail_hip(const char* what, hipError_t e) {
    fprintf(stderr, "teuk_run: %s: %s\n", what, hipGetErrorString(e));
    return 2;
}

static int fail_teuk(teuk_ctx* c, const char* what, int rc) {
    fprintf(stderr, "teuk_run: %s: %s (%s)\n", what, teuk_strerror(rc), c ? teuk_last_error(c) : "");
    return 2;
}

/* Copy n complex values between complex128 host data and the device state
 * of the chosen precision; tmp holds n complex64 values when prec is 32. */
static hipError_t upload(void* dev, const double* host, size_t n, int prec, float* tmp) {
    if (prec == TEUK_FP64) return hipMemcpy(dev, host, n * 16, hipMemcpyHostToDevice);
    for (size_t i = 0; i < 2 * n; ++i) tmp[i] = (float)host[i];
    return hipMemcpy(dev, tmp, n * 8, hipMemcpyHostToDevice);
}

static hipError_t download(double* host, const void* dev, size_t n, int prec, float* tmp) {
    if (prec == TEUK_FP64) return hipMemcpy(host, dev, n * 16, hipMemcpyDeviceToHost);
    hipError_t e = hipMemcpy(tmp, dev, n * 8, hipMemcpyDeviceToHost);
    for (size_t i = 0; i < 2 * n; ++i) host[i] = (double)tmp[i];
    return e;
}

int main(int argc, char** argv) {
    if (argc != 16 && argc != 17) {
        fprintf(stderr,
                "usage: %s IN OUT n_rstar n_theta rstar_min rstar_max a M m s dt r0 amp rstar_obs n_steps [prec]\n",
                argv[0]);
        return 1;
    }
    teuk_grid g;
    g.n_rstar = atoll(argv[3]);
    g.n_theta = atoll(argv[4]);
    g.rstar_min = atof(argv[5]);
    g.rstar_max = atof(argv[6]);
    const double a = atof(argv[7]), M = atof(argv[8]);
    const int m = atoi(argv[9]), s = atoi(argv[10]);
    const double dt = atof(argv[11]), r0 = atof(argv[12]), amp = atof(argv[13]), robs = atof(argv[14]);
    const long long n_steps = atoll(argv[15]);
    const int prec = argc == 17 ? atoi(argv[16]) : TEUK_FP64;
    if (g.n_rstar < 1 || g.n_theta < 1 || n_steps < 0 || (prec != TEUK_FP64 && prec != TEUK_FP32)) {
        fprintf(stderr, "teuk_run: bad sizes, step count or precision\n");
        return 1;
    }
    const size_t npts = (size_t)g.n_rstar * (size_t)g.n_theta;
    const size_t nwave = (size_t)(n_steps + 1) * (size_t)g.n_theta;
    const size_t es = prec == TEUK_FP64 ? 16 : 8;   /* bytes per complex value on the device */

    double* host = malloc(2 * npts * 16);
    double* wave_h = malloc(nwave * 16);
    float* tmp = malloc((npts > nwave ? npts : nwave) * 8);
    if (!host || !wave_h || !tmp) {
        fprintf(stderr, "teuk_run: host allocation failed\n");
        return 1;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f || fread(host, 16, 2 * npts, f) != 2 * npts) {
        fprintf(stderr, "teuk_run: cannot read %zu complex values from %s\n", 2 * npts, argv[1]);
        return 1;
    }
    fclose(f);

    void* buf[4] = {NULL, NULL, NULL, NULL};
    void* wave_d = NULL;
    hipError_t e;
    for (int i = 0; i < 4; ++i)
        if ((e = hipMalloc(&buf[i], npts * es)) != hipSuccess) return fail_hip("hipMalloc", e);
    if ((e = hipMalloc(&wave_d, nwave * es)) != hipSuccess) return fail_hip("hipMalloc", e);
    if ((e = upload(buf[0], host, npts, prec, tmp)) != hipSuccess) return fail_hip("upload Phi", e);
    if ((e = upload(buf[1], host + 2 * npts, npts, prec, tmp)) != hipSuccess) return fail_hip("upload Pi", e);

    teuk_ctx* c = NULL;
    int rc = teuk_create(&g, a, M, m, s, dt, prec, NULL, &c);
    if (rc != TEUK_OK) return fail_teuk(NULL, "teuk_create", rc);
    if ((rc = teuk_bind_state(c, buf[0], buf[1], buf[2], buf[3])) != TEUK_OK) return fail_teuk(c, "bind", rc);
    if (amp != 0.0 && (rc = teuk_set_source(c, r0, amp, 2.0, 2.0)) != TEUK_OK) return fail_teuk(c, "source", rc);
    if ((rc = teuk_set_observer(c, robs, wave_d, (int64_t)(n_steps + 1))) != TEUK_OK)
        return fail_teuk(c, "observer", rc);
    if ((rc = teuk_step(c, (int64_t)n_steps)) != TEUK_OK) return fail_teuk(c, "step", rc);
    if ((e = hipDeviceSynchronize()) != hipSuccess) return fail_hip("synchronize", e);
    if ((rc = teuk_check_finite(c)) != TEUK_OK) return fail_teuk(c, "check_finite", rc);
    const int cur = teuk_current(c);
    if (cur < 0) return fail_teuk(c, "current", cur);

    if ((e = download(host, buf[2 * cur], npts, prec, tmp)) != hipSuccess) return fail_hip("download Phi", e);
    if ((e = download(host + 2 * npts, buf[2 * cur + 1], npts, prec, tmp)) != hipSuccess)
        return fail_hip("download Pi", e);
    if ((e = download(wave_h, wave_d, nwave, prec, tmp)) != hipSuccess) return fail_hip("download wave", e);
    teuk_destroy(c);
    for (int i = 0; i < 4; ++i) (void)hipFree(buf[i]);
    (void)hipFree(wave_d);

    f = fopen(argv[2], "wb");
    if (!f || fwrite(host, 16, 2 * npts, f) != 2 * npts || fwrite(wave_h, 16, nwave, f) != nwave) {
        fprintf(stderr, "teuk_run: cannot write %s\n", argv[2]);
        return 1;
    }
    fclose(f);
    free(host);
    free(wave_h);
    free(tmp);
    return 0;
}
