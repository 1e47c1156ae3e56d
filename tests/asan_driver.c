/* C driver of the library's CPU-reachable paths (validation, status strings, NULL arguments, and
 * context and batch creation failing where no device is visible), run under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.  Prints one line per check. */
#include <stdio.h>
#include <string.h>
#include "snowlb.h"
int main(void) {
    snowlb_params p;
    const char* m = "";
    snowlb_params_default(&p);
    printf("validate default: %d\n", snowlb_validate(&p, NULL));
    for (int s = -7; s <= 1; ++s) printf("status %d: %s\n", s, snowlb_status_str(s));
    p.stencil = 3; printf("stencil 3: %d %s\n", snowlb_validate(&p, &m), m); p.stencil = 4;
    p.nx = 70000; printf("nx big: %d %s\n", snowlb_validate(&p, &m), m); p.nx = 128;
    snowlb_ctx* c = (snowlb_ctx*)0x1;
    printf("create NULL params: %d\n", snowlb_create(NULL, &c));
    printf("create valid (no GPU): %d ctx=%p err=%s\n", snowlb_create(&p, &c), (void*)c, snowlb_last_error(NULL));
    snowlb_destroy(NULL);
    printf("step NULL: %d\n", snowlb_step(NULL, 1, NULL));
    snowlb_params arr[2]; snowlb_params_default(&arr[0]); snowlb_params_default(&arr[1]); arr[1].flow = 1;
    snowlb_batch* b = (snowlb_batch*)0x1;
    printf("batch mixed: %d %s\n", snowlb_batch_create(arr, 2, &b), snowlb_batch_last_error(NULL));
    arr[1].flow = 0;
    printf("batch valid (no GPU): %d %s\n", snowlb_batch_create(arr, 2, &b), snowlb_batch_last_error(NULL));
    printf("tiles %d name0 %s name99 %s\n", snowlb_tile_count(), snowlb_tile_name(0), snowlb_tile_name(99));
    return 0;
}
