// Butcher tableaux of the three Runge--Kutta pairs, as compile-time constants
// for the kernels.  The paper names the methods (Section "Adaptive
// integration") without printing coefficients; they come from the primary
// publications:
//   Dopri5  Dormand & Prince (1980); continuous extension of Hairer, Norsett
//           & Wanner (1993, Sec. II.6)
//   Tsit5   Tsitouras (2011), with its interpolant
//   Verner7 Verner (2010), the 10-stage "efficient" 7(6) pair
// E(j) is the error weight b_j - bhat_j of eq:rk; B(j, q) gives the dense
// weights b_j(sigma) = sum_q B(j, q) sigma^(q+1) of eq:dense.
//
// All accessors are constexpr so that, inside the fully unrolled stage loops,
// every coefficient is an immediate and every zero coefficient disappears.
#pragma once

namespace gs {

struct Dopri5 {
  static constexpr int S = 7;
  static constexpr int ORDER = 5;
  static constexpr bool FSAL = true;
  static constexpr bool POLY_DENSE = true;
  static constexpr int DEG = 4;
  __host__ __device__ static constexpr double C(int j) {
    constexpr double v[7] = {0.0, 0.2, 0.3, 0.8, 8.0 / 9.0, 1.0, 1.0};
    return v[j];
  }
  __host__ __device__ static constexpr double A(int j, int l) {
    constexpr double v[7][7] = {
        {0, 0, 0, 0, 0, 0, 0},
        {1.0 / 5, 0, 0, 0, 0, 0, 0},
        {3.0 / 40, 9.0 / 40, 0, 0, 0, 0, 0},
        {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0, 0},
        {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0, 0},
        {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0, 0},
        {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0}};
    return v[j][l];
  }
  __host__ __device__ static constexpr double B(int j) { return A(6, j); }
  __host__ __device__ static constexpr double E(int j) {
    constexpr double v[7] = {71.0 / 57600, 0, -71.0 / 16695, 71.0 / 1920,
                             -17253.0 / 339200, 22.0 / 525, -1.0 / 40};
    return v[j];
  }
  __host__ __device__ static constexpr double Bs(int j, int q) {
    constexpr double v[7][4] = {
        {1.0, -8048581381.0 / 2820520608, 8663915743.0 / 2820520608,
         -12715105075.0 / 11282082432},
        {0, 0, 0, 0},
        {0, 131558114200.0 / 32700410799, -68118460800.0 / 10900136933,
         87487479700.0 / 32700410799},
        {0, -1754552775.0 / 470086768, 14199869525.0 / 1410260304,
         -10690763975.0 / 1880347072},
        {0, 127303824393.0 / 49829197408, -318862633887.0 / 49829197408,
         701980252875.0 / 199316789632},
        {0, -282668133.0 / 205662961, 2019193451.0 / 616988883, -1453857185.0 / 822651844},
        {0, 40617522.0 / 29380423, -110615467.0 / 29380423, 69997945.0 / 29380423}};
    return v[j][q];
  }
};

struct Tsit5 {
  static constexpr int S = 7;
  static constexpr int ORDER = 5;
  static constexpr bool FSAL = true;
  static constexpr bool POLY_DENSE = true;
  static constexpr int DEG = 4;
  __host__ __device__ static constexpr double C(int j) {
    constexpr double v[7] = {0.0, 0.161, 0.327, 0.9, 0.9800255409045097, 1.0, 1.0};
    return v[j];
  }
  __host__ __device__ static constexpr double A(int j, int l) {
    constexpr double v[7][7] = {
        {0, 0, 0, 0, 0, 0, 0},
        {0.161, 0, 0, 0, 0, 0, 0},
        {-0.008480655492356989, 0.335480655492357, 0, 0, 0, 0, 0},
        {2.897153057105493, -6.359448489975075, 4.3622954328695815, 0, 0, 0, 0},
        {5.325864828439257, -11.748883564062828, 7.4955393428898365, -0.09249506636175525, 0, 0,
         0},
        {5.86145544294642, -12.92096931784711, 8.159367898576159, -0.071584973281401,
         -0.028269050394068383, 0, 0},
        {0.09646076681806523, 0.01, 0.4798896504144996, 1.379008574103742, -3.290069515436081,
         2.324710524099774, 0}};
    return v[j][l];
  }
  __host__ __device__ static constexpr double B(int j) { return A(6, j); }
  __host__ __device__ static constexpr double E(int j) {
    constexpr double v[7] = {-0.00178001105222577714, -0.0008164344596567469,
                             0.007880878010261995,    -0.1447110071732629,
                             0.5823571654525552,      -0.45808210592918697,
                             0.015151515151515152};
    return v[j];
  }
  __host__ __device__ static constexpr double Bs(int j, int q) {
    constexpr double v[7][4] = {{1.0, -2.763706197274826, 2.9132554618219126, -1.0530884977290216},
                                {0, 0.13169999999999998, -0.2234, 0.1017},
                                {0, 3.9302962368947516, -5.941033872131505, 2.490627285651253},
                                {0, -12.411077166933676, 30.33818863028232, -16.548102889244902},
                                {0, 37.50931341651104, -88.1789048947664, 47.37952196281928},
                                {0, -27.896526289197286, 65.09189467479366, -34.8706578614966},
                                {0, 1.5, -4.0, 2.5}};
    return v[j][q];
  }
};

struct Verner7 {
  static constexpr int S = 10;
  static constexpr int ORDER = 7;
  static constexpr bool FSAL = false;
  static constexpr bool POLY_DENSE = false;  // outputs by a shortened step
  static constexpr int DEG = 0;
  __host__ __device__ static constexpr double C(int j) {
    constexpr double v[10] = {0.0,   0.005,
                              0.10888888888888888, 0.16333333333333333,
                              0.4555, 0.6095094489978381,
                              0.884, 0.925,
                              1.0,   1.0};
    return v[j];
  }
  __host__ __device__ static constexpr double A(int j, int l) {
    constexpr double v[10][10] = {
        {0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
        {0.005, 0, 0, 0, 0, 0, 0, 0, 0, 0},
        {-1.07679012345679, 1.185679012345679, 0, 0, 0, 0, 0, 0, 0, 0},
        {0.04083333333333333, 0, 0.1225, 0, 0, 0, 0, 0, 0, 0},
        {0.6389139236255726, 0, -2.455672638223657, 2.272258714598084, 0, 0, 0, 0, 0, 0},
        {-2.6615773750187572, 0, 10.804513886456137, -8.3539146573962, 0.820487594956657, 0, 0,
         0, 0, 0},
        {6.067741434696772, 0, -24.711273635911088, 20.427517930788895, -1.9061579788166472,
         1.006172249242068, 0, 0, 0, 0},
        {12.054670076253203, 0, -49.75478495046899, 41.142888638604674, -4.461760149974004,
         2.042334822239175, -0.09834843665406107, 0, 0, 0},
        {10.138146522881808, 0, -42.6411360317175, 35.76384003992257, -4.348022840392907,
         2.0098622683770357, 0.3487490460338272, -0.27143900510483127, 0, 0},
        {-45.030072034298676, 0, 187.3272437654589, -154.02882369350186, 18.56465306347536,
         -7.141809679295079, 1.3088085781613787, 0, 0, 0}};
    return v[j][l];
  }
  __host__ __device__ static constexpr double B(int j) {
    constexpr double v[10] = {0.04715561848627222,  0, 0, 0.25750564298434153,
                              0.26216653977412624,  0.15216092656738558,
                              0.49399691700324844,  -0.29430311714032503,
                              0.08131747232495111,  0};
    return v[j];
  }
  __host__ __device__ static constexpr double E(int j) {
    constexpr double v[10] = {0.002547011879931045, 0, 0, -0.00965839487279575,
                              0.04206470975639691,  -0.0666822437469301,
                              0.2650097464621281,   -0.29430311714032503,
                              0.08131747232495111,  -0.02029518466335628};
    return v[j];
  }
  __host__ __device__ static constexpr double Bs(int, int) { return 0.0; }
};

}  // namespace gs
