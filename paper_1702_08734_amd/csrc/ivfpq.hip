// IVFADC index: training, adding and searching (filled in below).
#include "common.hpp"

struct mk_ivfpq {
    int32_t d, nlist, M;
};

extern "C" mk_status mk_kmeans_assign(const float*, int64_t, int32_t, const float*, int32_t,
                                      int64_t*, float*, mk_stream_t) {
    MK_REQUIRE(false, MK_ERR_UNSUPPORTED, "not built yet");
}
extern "C" mk_status mk_kmeans_update(const float*, int64_t, int32_t, const int64_t*, int32_t,
                                      float*, int64_t*, mk_stream_t) {
    MK_REQUIRE(false, MK_ERR_UNSUPPORTED, "not built yet");
}
extern "C" mk_status mk_pq_encode(const float*, int64_t, int32_t, int32_t, const float*, uint8_t*,
                                  mk_stream_t) {
    MK_REQUIRE(false, MK_ERR_UNSUPPORTED, "not built yet");
}
extern "C" mk_status mk_ivfpq_create(int32_t, int32_t, int32_t, mk_ivfpq**) {
    MK_REQUIRE(false, MK_ERR_UNSUPPORTED, "not built yet");
}
extern "C" void mk_ivfpq_destroy(mk_ivfpq* p) { delete p; }
extern "C" mk_status mk_ivfpq_train(mk_ivfpq*, const float*, int64_t, int32_t, const int64_t*,
                                    const int64_t*, mk_stream_t) {
    MK_REQUIRE(false, MK_ERR_UNSUPPORTED, "not built yet");
}
extern "C" mk_status mk_ivfpq_add(mk_ivfpq*, const float*, int64_t, mk_stream_t) {
    MK_REQUIRE(false, MK_ERR_UNSUPPORTED, "not built yet");
}
extern "C" int64_t mk_ivfpq_ntotal(const mk_ivfpq*) { return 0; }
extern "C" mk_status mk_ivfpq_search(mk_ivfpq*, const float*, int64_t, int32_t, int32_t, float*,
                                     int64_t*, mk_stream_t) {
    MK_REQUIRE(false, MK_ERR_UNSUPPORTED, "not built yet");
}
extern "C" mk_status mk_ivfpq_get_quantizers(const mk_ivfpq*, float*, float*) {
    MK_REQUIRE(false, MK_ERR_UNSUPPORTED, "not built yet");
}
extern "C" mk_status mk_ivfpq_set_quantizers(mk_ivfpq*, const float*, const float*, mk_stream_t) {
    MK_REQUIRE(false, MK_ERR_UNSUPPORTED, "not built yet");
}
extern "C" mk_status mk_ivfpq_get_lists(const mk_ivfpq*, int64_t*, uint8_t*, int64_t*) {
    MK_REQUIRE(false, MK_ERR_UNSUPPORTED, "not built yet");
}
