/* Bootstrapping for the oracle (test infrastructure only). */
#include <stddef.h>
typedef struct orc_ctx orc_ctx;
typedef struct orc_ct orc_ct;
orc_ct *orc_bootstrap(orc_ctx *c, const orc_ct *a) { (void)c; (void)a; return NULL; }
