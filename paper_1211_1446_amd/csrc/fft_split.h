// (A, B) splits of the FFT lengths that have compiled two-step kernels (the
// same tables as fft2::dispatch_plane / dispatch_z), and the scrambled-position
// -> natural-index map of their real-space output.
#pragma once

namespace dks {
namespace fft2 {

inline bool split_lookup(const int (*tab)[3], int count, int n, int *A, int *B) {
  for (int i = 0; i < count; ++i)
    if (tab[i][0] == n) {
      *A = tab[i][1];
      *B = tab[i][2];
      return true;
    }
  return false;
}

// plane axes (a1, a2): n <= 128
inline bool split_plane(int n, int *A, int *B) {
  static const int tab[][3] = {
      {8, 1, 8},    {9, 1, 9},    {10, 1, 10},  {12, 1, 12},   {15, 1, 15}, {16, 1, 16},
      {18, 3, 6},   {20, 4, 5},   {24, 4, 6},   {25, 5, 5},    {27, 3, 9},  {30, 5, 6},
      {32, 4, 8},   {36, 6, 6},   {40, 5, 8},   {45, 5, 9},    {48, 6, 8},  {50, 5, 10},
      {54, 6, 9},   {60, 6, 10},  {64, 8, 8},   {72, 8, 9},    {75, 5, 15}, {80, 8, 10},
      {90, 9, 10},  {96, 8, 12},  {100, 10, 10}, {120, 10, 12}, {128, 8, 16}};
  return split_lookup(tab, (int)(sizeof(tab) / sizeof(tab[0])), n, A, B);
}

// z lines (a3): the plane lengths and larger ones up to 400
inline bool split_z(int n, int *A, int *B) {
  static const int tab[][3] = {{144, 12, 12}, {160, 10, 16}, {180, 12, 15}, {192, 12, 16},
                               {200, 10, 20}, {240, 15, 16}, {256, 16, 16}, {288, 16, 18},
                               {320, 16, 20}, {360, 18, 20}, {400, 20, 20}};
  if (split_plane(n, A, B)) return true;
  return split_lookup(tab, (int)(sizeof(tab) / sizeof(tab[0])), n, A, B);
}

// scrambled real-space position p -> natural index j (both in [0, n))
inline int scrambled_to_natural(int p, int A, int B) {
  const int ka = p / B, kb = p % B;
  return ka + A * kb;
}

}  // namespace fft2
}  // namespace dks
