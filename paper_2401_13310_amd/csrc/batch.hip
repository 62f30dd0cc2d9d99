// batch.hip -- batched filling of many histograms (placeholder until the
// persistent kernel lands).
#include "plan.h"

using namespace hg;

struct hist_batch_s {
    int k = 0;
};

extern "C" hist_status hist_batch_create(int k, hist_t *const *hs, const hist_fill_desc *descs,
                                         hist_batch_t **out, void *stream)
{
    (void)k; (void)hs; (void)descs; (void)stream;
    if (out)
        *out = nullptr;
    return set_error(HIST_ENOTSUP, "hist_batch_create: not available yet");
}

extern "C" hist_status hist_batch_launch(hist_batch_t *b, void *stream)
{
    (void)b; (void)stream;
    return set_error(HIST_ENOTSUP, "hist_batch_launch: not available yet");
}

extern "C" hist_status hist_batch_launch_eager(hist_batch_t *b, void *stream)
{
    (void)b; (void)stream;
    return set_error(HIST_ENOTSUP, "hist_batch_launch_eager: not available yet");
}

extern "C" hist_status hist_batch_destroy(hist_batch_t *b)
{
    delete b;
    return HIST_OK;
}
