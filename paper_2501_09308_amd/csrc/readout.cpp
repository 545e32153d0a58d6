// Posterior readout of a converged analysis: expected weights, their
// standard deviations, area ratios and the threshold selection of phases
// (Sec. 4: the phases whose area ratio exceeds 1 % are the identified ones).
#include <cmath>
#include <string>
#include <vector>

#include "xrdvi.h"

namespace xrdvi {
void set_error(const std::string &msg);
}

extern "C" int xrdvi_readout(int32_t K, const int32_t *peak_off,
                             const double *peak_int, const double *loc_h,
                             const double *logscale_h, double threshold,
                             double *mean_h, double *sd_h, double *area_ratio,
                             int32_t *selected) {
    try {
        if (K < 1 || !peak_off || !loc_h || !logscale_h) {
            xrdvi::set_error("readout: K >= 1 and non-NULL peak_off, loc_h, logscale_h required");
            return XRDVI_EINVAL;
        }
        if (!(threshold >= 0.0 && threshold < 1.0)) {
            xrdvi::set_error("readout: threshold must lie in [0, 1)");
            return XRDVI_EINVAL;
        }
        if (peak_off[0] != 0 || (peak_off[K] > 0 && !peak_int)) {
            xrdvi::set_error("readout: peak_off[0] must be 0 and peak_int non-NULL");
            return XRDVI_EINVAL;
        }
        for (int k = 0; k < K; ++k) {
            if (peak_off[k + 1] < peak_off[k]) {
                xrdvi::set_error("readout: peak_off must be non-decreasing");
                return XRDVI_EINVAL;
            }
            if (!std::isfinite(loc_h[k]) || !std::isfinite(logscale_h[k])) {
                xrdvi::set_error("readout: loc_h and logscale_h must be finite");
                return XRDVI_EINVAL;
            }
        }
        // area_k = E[h_k] * sum_m I_m with E[h] of the log-normal q(h)
        std::vector<double> area(K);
        double total = 0.0;
        for (int k = 0; k < K; ++k) {
            const double s2 = std::exp(2.0 * logscale_h[k]);
            const double m = std::exp(loc_h[k] + 0.5 * s2);
            double isum = 0.0;
            for (int j = peak_off[k]; j < peak_off[k + 1]; ++j) isum += peak_int[j];
            if (mean_h) mean_h[k] = m;
            if (sd_h) sd_h[k] = m * std::sqrt(std::expm1(s2));
            area[k] = m * isum;
            total += area[k];
        }
        if (!(total > 0.0) || !std::isfinite(total)) {
            xrdvi::set_error("readout: the total area must be positive and finite");
            return XRDVI_EINVAL;
        }
        for (int k = 0; k < K; ++k) {
            const double ratio = area[k] / total;
            if (area_ratio) area_ratio[k] = ratio;
            if (selected) selected[k] = ratio > threshold ? 1 : 0;
        }
        return XRDVI_OK;
    } catch (...) {
        xrdvi::set_error("readout: unexpected internal exception");
        return XRDVI_EDEVICE;
    }
}
