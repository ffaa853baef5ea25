// vmc_mass_start.hpp -- written by paper_1010_2107_amd/gen_mass_start.py; do not edit.
//
// Start of the Newton inversion of the RAMBO-on-diet mass fraction CDF
// F(t) = (k+1) t^k - k t^(k+1): v ~ s rho(s), with v = t, s = (r/(k+1))^(1/k)
// for r < 1/2 and v = 1 - t, s = sqrt(2 (1 - r) / (k (k+1))) otherwise;
// rho is a degree-5 polynomial fitted to v / s (coefficients by ascending
// power, rows k = 2..4).
//   k=2: start max rel err 2.51e-05; after one FP32 Newton step t 1.52e-07, u 1.46e-07
//   k=3: start max rel err 7.75e-05; after one FP32 Newton step t 1.30e-07, u 1.69e-07
//   k=4: start max rel err 1.45e-04; after one FP32 Newton step t 1.19e-07, u 1.89e-07
#pragma once

namespace vmc {

constexpr int kMassStartDeg = 5;
constexpr int kMassStartMinK = 2;
constexpr int kMassStartMaxK = 4;
constexpr double kMassStartLo[3][6] = {
    {9.99975437840538550e-01, 3.37235623205481005e-01, 1.78801282476558326e-01, 1.18430858640364756e+00, -2.99660367886487933e+00, 5.28381196422735755e+00},  // k = 2
    {9.99924191352309699e-01, 2.59566925208408406e-01, -5.10335787324863854e-03, 1.54913226055412068e+00, -3.84777067870052392e+00, 4.69958676464518277e+00},  // k = 3
    {9.99858553626873814e-01, 2.15570210161169257e-01, -1.33395357775947188e-01, 1.81725737089185269e+00, -4.20402698749091819e+00, 4.23951170873022409e+00},  // k = 4
};
constexpr double kMassStartHi[3][6] = {
    {9.99975438611396261e-01, 3.37235514090877098e-01, 1.78803706447344224e-01, 1.18429001295561309e+00, -2.99654625096968052e+00, 5.28375038766540506e+00},  // k = 2
    {9.99954726429939988e-01, 6.76926519679483585e-01, 4.90949583081102092e-01, 6.08412971961362015e+00, -2.27855967211897728e+01, 5.57346477747324727e+01},  // k = 3
    {9.99939506043021731e-01, 1.01778415512139997e+00, 9.18895577212430759e-01, 1.73926065791455038e+01, -8.60055186552607722e+01, 2.69054299008667101e+02},  // k = 4
};

}  // namespace vmc
