// Host-side check of the transpose table's size grouping (launch.h): for
// element-size lists read from the command line, prints the order and the
// group ends, one line each.
#include <stdio.h>
#include <stdlib.h>

#include "launch.h"

int main(int argc, char** argv) {
  soax::XposeArgs t{};
  t.narrays = argc - 1;
  for (int a = 0; a < t.narrays; ++a) t.es[a] = atoi(argv[a + 1]);
  soax::group_by_size(t);
  for (int a = 0; a < t.narrays; ++a) printf("%d ", t.order[a]);
  printf("\n%d %d %d\n", t.group_end[0], t.group_end[1], t.group_end[2]);
  return 0;
}
