// axpic_tables.h -- host builders of the thermal-channel quantile tables.
#pragma once

namespace axpic_host {
constexpr int kTabN = 3072;
constexpr double kTabZ0 = -18.0, kTabZ1 = 36.0;
// tab has 2 (kTabN + 1) doubles: y = ln x at the nodes, then dy/dz.
void build_compton_table(double* tab);
void build_gamma_table(double* tab, double k);
}  // namespace axpic_host
