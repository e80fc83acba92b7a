/* Plain C caller of the library's host-only entry points (no GPU needed):
 * prints the characteristic polynomial of xoshiro256 and x^J mod p for the
 * jump and long jump, as hexadecimal words, for comparison with the oracle. */
#include <stdio.h>
#include <stdint.h>

#include "slrng.h"

int main(void) {
  uint64_t p[5], r[4];
  if (slrng_version() != SLRNG_ABI_VERSION) return 2;
  if (slrng_state_words(SLRNG_XOSHIRO256_STARSTAR) != 4) return 3;
  if (slrng_charpoly(SLRNG_XOSHIRO256_STARSTAR, p, 5) != SLRNG_OK) return 4;
  printf("charpoly");
  for (int i = 0; i < 5; i++) printf(" %016llx", (unsigned long long)p[i]);
  printf("\n");
  const uint64_t jump[3] = {0, 0, 1};  /* 2^128 */
  const uint64_t longjump[4] = {0, 0, 0, 1};  /* 2^192 */
  if (slrng_jump_poly(SLRNG_XOSHIRO256_STARSTAR, jump, 3, r, 4) != SLRNG_OK) return 5;
  printf("jump");
  for (int i = 0; i < 4; i++) printf(" %016llx", (unsigned long long)r[i]);
  printf("\n");
  if (slrng_jump_poly(SLRNG_XOSHIRO256_STARSTAR, longjump, 4, r, 4) != SLRNG_OK) return 6;
  printf("longjump");
  for (int i = 0; i < 4; i++) printf(" %016llx", (unsigned long long)r[i]);
  printf("\n");
  /* errors are return codes, never exceptions */
  if (slrng_charpoly(99, p, 5) != SLRNG_EINVAL) return 7;
  if (slrng_streams_jump(NULL, SLRNG_JUMP, NULL) != SLRNG_EINVAL) return 8;
  printf("%s\n", slrng_strerror(SLRNG_EZEROSTATE));
  return 0;
}
