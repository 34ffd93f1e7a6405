// placeholder while the estimator is written
#include "saba_internal.hpp"
using namespace saba;
extern "C" int saba_aesc(saba_graph *, const saba_aesc_params *, double *, saba_stats *, void *) { set_error("not built"); return SABA_E_INVALID; }
extern "C" int saba_aesc_query(saba_graph *, const saba_aesc_params *, const int32_t *, int64_t, double *, saba_stats *, void *) { set_error("not built"); return SABA_E_INVALID; }
extern "C" int saba_aesc_edge_stats(saba_graph *, const saba_aesc_params *, double *, int32_t *, int32_t *, int64_t *, double *, double *, int64_t *, int64_t *, double *, saba_stats *, void *) { set_error("not built"); return SABA_E_INVALID; }
