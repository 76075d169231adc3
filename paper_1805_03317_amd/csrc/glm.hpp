// Per-observation control-variate remainder d = l_k - q_k and its derivative
// d' with respect to the linear predictor (section 3.2: q_k is the Taylor
// expansion of l_k around theta_bar; gradient of d_k is d' x_k).
//
// Everything is evaluated from the per-row constants stored next to x_k:
//   eta_bar = x_k' theta_bar and aux = sigmoid(-|eta_bar|) (logistic),
//   exp(eta_bar) (Poisson) or y_k - eta_bar (Student-t), plus
//   Delta = x_k' (theta - theta_bar).
// The remainder is O(Delta^3) while l_k is O(1), so it is never formed as a
// difference of the two: each family uses an expansion whose terms are of the
// size of the result.
//
// Logistic, l(eta) = y eta - softplus(eta): the y terms cancel exactly and
//   d = -R, d' = -R' with R the second-order Taylor remainder of softplus.
//   softplus(x) = x + softplus(-x), so R(eta_bar, Delta) = R(-eta_bar, -Delta)
//   and the evaluation always runs with s = sigmoid(eta_bar) <= 1/2.
//   softplus(eta_bar + t) - softplus(eta_bar) = log(1 - s + s e^t) is the
//   cumulant generating function of a Bernoulli(s) variable, so for small
//   |Delta| R = sum_{k>=3} kappa_k Delta^k / k! with the Bernoulli cumulants
//   kappa_k = v P_k(v) (k even) or v (1-2s) P_k(v) (k odd), v = s(1-s), from
//   the recursion kappa_{k+1} = v d(kappa_k)/ds.
//   Medium |Delta| uses R = L3(z) + s E3 - s^2 Delta E2 - s^2 E2^2 / 2 with
//   z = s expm1(Delta), E2 = e^D - 1 - D, E3 = E2 - D^2/2, L3(z) = log1p(z) - z + z^2/2;
//   large |Delta| uses the softplus difference directly.
// Poisson, l = y eta - e^eta - log y!: d = -e^{eta_bar} E3(Delta),
//   d' = -e^{eta_bar} E2(Delta).
// Student-t (t_5 errors), l = -(nu+1)/2 log(1 + r^2/nu) + const, r = y - eta:
//   with r_bar = y - eta_bar (stored as aux), s = nu + r_bar^2,
//   z = Delta (Delta - 2 r_bar) / s and t = nu + (r_bar - Delta)^2 = s (1 + z),
//   d = (nu+1) [Delta^3 (Delta/4 - r_bar) / s^2 - L3(z)/2],
//   d' = (nu+1) Delta^2 [r_bar (r_bar^2 - 3 nu) - Delta (r_bar^2 - nu)] / (s^2 t),
//   the second-order terms cancelling exactly in both.
// Gaussian (known variance, test family): d = d' = 0 exactly.
// First-order control variate (cv_order 1): the dropped f'' Delta^2 / 2 term
// is added back: d1 = d2 + f''(eta_bar) Delta^2 / 2, d1' = d2' + f''(eta_bar) Delta.
#pragma once
#include <hip/hip_runtime.h>

namespace subsmc {

enum Family : int { kLogistic = 0, kPoisson = 1, kGaussian = 2, kStudentT = 3 };

// Student-t regression (Experiment 2): e ~ t_nu with nu = 5 and unit scale.
constexpr double kStudentNu = 5.0;

template <typename T> struct Tol;
template <> struct Tol<double> {
  static constexpr double series_logistic = 0.25;  // |Delta| below: cumulant series
  static constexpr double direct_logistic = 2.0;   // |Delta| above: softplus difference
  static constexpr double series_exp = 0.5;         // |Delta| below: exp series for E2/E3
  static constexpr int n_cumulant = 14;
  static constexpr int n_exp = 16;
};
template <> struct Tol<float> {
  // FP32 rows: the cumulant series up to |Delta| = 1.25. The log1p form below
  // adds terms of order Delta^3 whose sum is of order Delta^4 near s = 1/2
  // (kappa_3 = 0 there), which in FP32 costs up to ~1e-4 of the result for
  // |Delta| in [0.25, 1); the series has no such cancellation. Its terms fall
  // like (|Delta| / pi)^k (the nearest singularity of log(1 - s + s e^t) is at
  // |t| >= pi), so 8, 12 and 16 terms reach FP32 rounding for |Delta| below
  // 0.3, 0.7 and 1.25.
  static constexpr float series_logistic = 1.25f;
  static constexpr float direct_logistic = 2.0f;
  static constexpr float series_exp = 1.0f;
  static constexpr float series_short = 0.3f;
  static constexpr float series_mid = 0.7f;
  static constexpr int n_cumulant = 16;
  static constexpr int n_short = 8;
  static constexpr int n_mid = 12;
  static constexpr int n_exp = 12;
};

__device__ __forceinline__ double dev_expm1(double x) { return expm1(x); }
__device__ __forceinline__ float dev_expm1(float x) { return expm1f(x); }
__device__ __forceinline__ double dev_log1p(double x) { return log1p(x); }
__device__ __forceinline__ float dev_log1p(float x) { return log1pf(x); }
__device__ __forceinline__ double dev_exp(double x) { return exp(x); }
__device__ __forceinline__ float dev_exp(float x) { return expf(x); }

template <typename T>
__device__ __forceinline__ T softplus(T x) {
  const T ax = x < T(0) ? -x : x;
  return (x > T(0) ? x : T(0)) + dev_log1p(dev_exp(-ax));
}

template <typename T>
__device__ __forceinline__ T sigmoid(T x) {
  if (x >= T(0)) return T(1) / (T(1) + dev_exp(-x));
  const T e = dev_exp(x);
  return e / (T(1) + e);
}

// Bernoulli cumulant kappa_k(s), k = 3..16, as v P_k(v) (k even) or
// v (1 - 2s) P_k(v) (k odd), v = s (1 - s), w = 1 - 2s; the integer
// coefficients of P_k (ascending powers of v) follow from
// kappa_{k+1} = v d(kappa_k)/ds with kappa_1 = s.
template <typename T>
__device__ __forceinline__ T cumulant(int k, T v, T w) {
  T p;
  switch (k) {
    case 3: p = T(1); break;
    case 4: p = T(1) + v * T(-6); break;
    case 5: p = T(1) + v * T(-12); break;
    case 6: p = T(1) + v * (T(-30) + v * T(120)); break;
    case 7: p = T(1) + v * (T(-60) + v * T(360)); break;
    case 8: p = T(1) + v * (T(-126) + v * (T(1680) + v * T(-5040))); break;
    case 9: p = T(1) + v * (T(-252) + v * (T(5040) + v * T(-20160))); break;
    case 10: p = T(1) + v * (T(-510) + v * (T(17640) + v * (T(-151200) + v * T(362880)))); break;
    case 11: p = T(1) + v * (T(-1020) + v * (T(52920) + v * (T(-604800) + v * T(1814400)))); break;
    case 12:
      p = T(1) + v * (T(-2046) + v * (T(168960) + v * (T(-3160080) + v * (T(19958400) + v * T(-39916800)))));
      break;
    case 13:
      p = T(1) + v * (T(-4092) + v * (T(506880) + v * (T(-12640320) + v * (T(99792000) + v * T(-239500800)))));
      break;
    case 14:
      p = T(1) + v * (T(-8190) + v * (T(1561560) + v * (T(-57657600) +
              v * (T(726485760) + v * (T(-3632428800.0) + v * T(6227020800.0))))));
      break;
    case 15:
      p = T(1) + v * (T(-16380) + v * (T(4684680) + v * (T(-230630400) +
              v * (T(3632428800.0) + v * (T(-21794572800.0) + v * T(43589145600.0))))));
      break;
    default:
      p = T(1) + v * (T(-32766) + v * (T(14217840) + v * (T(-988107120) + v * (T(22313491200.0) +
              v * (T(-210680870400.0) + v * (T(871782912000.0) + v * T(-1307674368000.0)))))));
      break;
  }
  return (k & 1) ? v * w * p : v * p;
}

// 1/k! for k = 0..16
template <typename T>
__device__ __forceinline__ T inv_fact(int k) {
  switch (k) {
    case 0: case 1: return T(1);
    case 2: return T(0.5);
    case 3: return T(1.0 / 6.0);
    case 4: return T(1.0 / 24.0);
    case 5: return T(1.0 / 120.0);
    case 6: return T(1.0 / 720.0);
    case 7: return T(1.0 / 5040.0);
    case 8: return T(1.0 / 40320.0);
    case 9: return T(1.0 / 362880.0);
    case 10: return T(1.0 / 3628800.0);
    case 11: return T(1.0 / 39916800.0);
    case 12: return T(1.0 / 479001600.0);
    case 13: return T(1.0 / 6227020800.0);
    case 14: return T(1.0 / 87178291200.0);
    case 15: return T(1.0 / 1307674368000.0);
    default: return T(1.0 / 20922789888000.0);
  }
}

// e^D - 1 for |D| >= 1 in FP32: e^D = 2^t (1 + ln2 r) with t = D log2(e)
// rounded and r its rounding error (an FMA plus the low part of log2(e)),
// 2^t from the hardware exponential; about 2 ulp, and for |D| >= 1 the
// subtraction of 1 loses at most 1.3 bits.
__device__ __forceinline__ float exp_minus_one_wide(float D) {
  constexpr float kL2eHi = 1.44269502162933349609375f;   // log2(e) rounded to float
  constexpr float kL2eLo = 1.925963033500011079e-8f;     // log2(e) - kL2eHi
  constexpr float kLn2 = 0.693147180559945309f;
  const float t = D * kL2eHi;
  const float r = __builtin_fmaf(D, kL2eHi, -t) + D * kL2eLo;
  const float p = __builtin_amdgcn_exp2f(t);
  return __builtin_fmaf(p, kLn2 * r, p) - 1.0f;
}

// E2 = e^D - 1 - D and E3 = e^D - 1 - D - D^2/2: the Taylor series below
// |D| = series_exp, e^D - 1 beyond. Every lane evaluates the series (no
// change of the execution mask, so the series schedules together with the
// surrounding arithmetic); the exponential branch runs only when some lane of
// the wavefront needs it (NB: on every lane, without a branch), and each lane
// keeps the result of its own branch.
template <typename T, bool NB = false>
__device__ __forceinline__ void exp_remainders(T D, T& E2, T& E3) {
  const T aD = D < T(0) ? -D : D;
  T acc = T(0);
#pragma unroll
  for (int k = Tol<T>::n_exp; k >= 3; --k) acc = acc * D + inv_fact<T>(k);
  E3 = acc * D * D * D;
  E2 = E3 + T(0.5) * D * D;
  const bool wide = !(aD < Tol<T>::series_exp);  // NaN takes this branch too
  if (NB || __any(wide)) {
    T em1;
    if constexpr (sizeof(T) == 4) em1 = exp_minus_one_wide(D);
    else em1 = dev_expm1(D);
    const T E2w = em1 - D;
    const T E3w = E2w - T(0.5) * D * D;
    E2 = wide ? E2w : E2;
    E3 = wide ? E3w : E3;
  }
}

// R = sum_{k=3..K} kappa_k D^k / k! and R' = sum_{k=3..K} kappa_k D^(k-1) / (k-1)!
template <typename T, int K>
__device__ __forceinline__ void cumulant_series(T v, T w, T D, T& R, T& Rp) {
  T r = T(0), rp = T(0);
#pragma unroll
  for (int k = K; k >= 3; --k) {
    const T c = cumulant<T>(k, v, w);
    r = r * D + c * inv_fact<T>(k);
    rp = rp * D + c * inv_fact<T>(k - 1);
  }
  R = r * D * D * D;
  Rp = rp * D * D;
}

// Second-order Taylor remainder of softplus at eta_bar <= 0 (s = sigmoid(eta_bar)).
template <typename T>
__device__ __forceinline__ void softplus_remainder(T eb, T s, T D, T& R, T& Rp) {
  const T sc = T(1) - s;
  const T v = s * sc;
  const T w = sc - s;
  const T aD = D < T(0) ? -D : D;
  if constexpr (sizeof(T) == 4) {
    // the number of series terms follows the largest |D| of the wavefront
    // (a uniform branch); lanes beyond the series range take their own branch
    if (!__any(!(aD < Tol<T>::series_short))) {
      cumulant_series<T, Tol<T>::n_short>(v, w, D, R, Rp);
      return;
    }
    if (!__any(!(aD < Tol<T>::series_mid))) {
      cumulant_series<T, Tol<T>::n_mid>(v, w, D, R, Rp);
      return;
    }
  }
  if (aD < Tol<T>::series_logistic) {
    cumulant_series<T, Tol<T>::n_cumulant>(v, w, D, R, Rp);
  } else if (aD <= Tol<T>::direct_logistic) {
    const T em1 = dev_expm1(D);
    const T E2 = em1 - D;
    const T E3 = E2 - T(0.5) * D * D;
    const T z = s * em1;
    const T L3 = dev_log1p(z) - z + T(0.5) * z * z;
    R = L3 + s * E3 - s * s * D * E2 - T(0.5) * s * s * E2 * E2;
    Rp = v * (T(0.5) * w * D * D + E3 - s * D * E2) / (T(1) + z);
  } else {
    const T sp0 = -dev_log1p(-s);  // softplus(eb) for eb <= 0
    R = (softplus<T>(eb + D) - sp0) - s * D - T(0.5) * v * D * D;
    Rp = (sigmoid<T>(eb + D) - s) - v * D;
  }
}

// L3(z) = log1p(z) - z + z^2/2 = sum_{k>=3} (-1)^(k+1) z^k / k, z > -1
template <typename T>
__device__ __forceinline__ T log1p_remainder3(T z) {
  constexpr T kSeries = sizeof(T) == 4 ? T(0.25) : T(0.125);
  constexpr int kTerms = sizeof(T) == 4 ? 15 : 22;
  const T az = z < T(0) ? -z : z;
  if (az < kSeries) {
    T acc = T(0);
#pragma unroll
    for (int k = kTerms; k >= 3; --k) acc = acc * z + ((k & 1) ? T(1) : T(-1)) / T(k);
    return acc * z * z * z;
  }
  return dev_log1p(z) - z + T(0.5) * z * z;
}

// Returns d (remainder) and dp (its eta-derivative); FAM is the family. NB:
// the Poisson remainder without a branch (its exponential form evaluated on
// every lane), so that it forms one block with the work around it.
template <typename T, int FAM, bool NB = false>
__device__ __forceinline__ void cv_remainder(int cv_order, T eb, T aux, T D, T inv_s2, T& d, T& dp) {
  if constexpr (FAM == kLogistic) {
    const bool flip = eb > T(0);
    const T e = flip ? -eb : eb;
    const T Dm = flip ? -D : D;
    T R, Rp;
    softplus_remainder<T>(e, aux, Dm, R, Rp);
    d = -R;
    dp = flip ? Rp : -Rp;
    if (cv_order == 1) {
      const T v = aux * (T(1) - aux);
      d -= T(0.5) * v * D * D;
      dp -= v * D;
    }
  } else if constexpr (FAM == kPoisson) {
    T E2, E3;
    exp_remainders<T, NB>(D, E2, E3);
    d = -aux * E3;
    dp = -aux * E2;
    if (cv_order == 1) {
      d -= T(0.5) * aux * D * D;
      dp -= aux * D;
    }
  } else if constexpr (FAM == kStudentT) {
    const T nu = T(kStudentNu);
    const T rb = aux;
    const T rb2 = rb * rb;
    const T s = nu + rb2;
    const T is = T(1) / s;
    const T z = D * (D - T(2) * rb) * is;
    const T tt = nu + (rb - D) * (rb - D);
    const T D2 = D * D;
    d = (nu + T(1)) * (D2 * D * (T(0.25) * D - rb) * is * is - T(0.5) * log1p_remainder3<T>(z));
    dp = (nu + T(1)) * D2 * (rb * (rb2 - T(3) * nu) - D * (rb2 - nu)) * is * is / tt;
    if (cv_order == 1) {
      const T f2 = (nu + T(1)) * (rb2 - nu) * is * is;
      d += T(0.5) * f2 * D2;
      dp += f2 * D;
    }
  } else {
    d = T(0);
    dp = T(0);
    if (cv_order == 1) {
      d = -T(0.5) * inv_s2 * D * D;
      dp = -inv_s2 * D;
    }
  }
}

// Full-data log-density and its first two eta-derivatives (FP64), for the
// control-variate summaries A, B, C.
// l_k and its first two eta-derivatives, without the terms that do not
// depend on eta (log y! for Poisson, log(2 pi s2)/2 for Gaussian): those are
// summed once by loglik_const.
__device__ __forceinline__ void loglik_derivs(int family, double y, double eta, double inv_s2,
                                              double& f0, double& f1, double& f2) {
  if (family == kLogistic) {
    const double s = sigmoid<double>(eta);
    const double sn = sigmoid<double>(-eta);
    f0 = y * eta - softplus<double>(eta);
    f1 = y - s;
    f2 = -s * sn;
  } else if (family == kPoisson) {
    const double mu = exp(eta);
    f0 = y * eta - mu;
    f1 = y - mu;
    f2 = -mu;
  } else if (family == kStudentT) {
    const double r = y - eta, t = kStudentNu + r * r;
    f0 = -0.5 * (kStudentNu + 1.0) * log1p(r * r / kStudentNu);
    f1 = (kStudentNu + 1.0) * r / t;
    f2 = (kStudentNu + 1.0) * (r * r - kStudentNu) / (t * t);
  } else {
    const double r = y - eta;
    f0 = -0.5 * r * r * inv_s2;
    f1 = r * inv_s2;
    f2 = -inv_s2;
  }
}

__device__ __forceinline__ double loglik_const(int family, double y, double log2pis2) {
  if (family == kPoisson) return -lgamma(y + 1.0);
  if (family == kStudentT)
    return lgamma(0.5 * (kStudentNu + 1.0)) - lgamma(0.5 * kStudentNu) - 0.5 * log(kStudentNu * M_PI);
  if (family == kGaussian) return -0.5 * log2pis2;
  return 0.0;
}

}  // namespace subsmc
