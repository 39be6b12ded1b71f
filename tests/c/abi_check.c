/* Host-only use of the C ABI from plain C: every call here validates its
 * arguments or reports sizes before any device work, so it runs without a
 * GPU.  Prints one "name value" line per check for the test to compare. */
#include <stdio.h>
#include <string.h>

#include "fewbody.h"

int main(void)
{
    printf("version_has_gfx950 %d\n", strstr(fb_version(), "gfx950") != NULL);

    fb_opts o;
    fb_opts_default(&o);
    printf("opts_default %d %g %d %g %d\n", o.adaptive, o.eta, o.stop_rules, o.r_eject, o.schedule);

    const int32_t nb_ok[3] = {3, 5, 40};
    const int32_t nb_bad[2] = {3, 1};
    printf("workspace_ok %d\n", fb_workspace_bytes(3, nb_ok) > 0);
    printf("workspace_bad %zu\n", fb_workspace_bytes(2, nb_bad));

    printf("log_rv %zu\n", fb_log_bytes(3, nb_ok, FB_LOG_RV, 4));
    printf("log_state %zu\n", fb_log_bytes(3, nb_ok, FB_LOG_STATE, 4));
    printf("log_bad_kind %zu\n", fb_log_bytes(3, nb_ok, 7, 4));

    printf("integrate_null %d\n", (int)fb_integrate_steps(NULL, 10, 0.1, NULL));
    printf("last_error_set %d\n", fb_last_error() != NULL && fb_last_error()[0] != '\0');

    const double m[2] = {1.0, 1e-3};
    const double x[6] = {0, 0, 0, 1, 0, 0};
    const double v[6] = {0, 0, 0, 0, 1, 0};
    const int32_t one[1] = {1};
    fb_ensemble *e = NULL;
    printf("create_bad_n %d %d\n", (int)fb_ensemble_create(1, one, m, x, v, NULL, NULL, &e), e == NULL);

    fb_server_opts so;
    fb_server_opts_default(&so);
    printf("server_request_ok %d\n", fb_server_request_bytes(&so, 2, nb_ok) > 0);
    printf("server_request_large %zu\n", fb_server_request_bytes(&so, 3, nb_ok));
    so.idle_spread = 5;
    printf("server_bad_spread %zu\n", fb_server_request_bytes(&so, 2, nb_ok));
    printf("sizes %zu %zu\n", sizeof(fb_server_opts), sizeof(fb_server_stats));
    return 0;
}
