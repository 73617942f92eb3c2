/*
 * qm_table.cpp -- host builder of the normal -> Student t tables.
 */
#include <cstdio>
#include "qm_table.h"

namespace qm {
int build_student_table(double nu, HostTTable* out, char* err, int errlen)
{
    (void)nu; (void)out;
    snprintf(err, errlen, "not available in this build");
    return -1;
}
void free_student_table(HostTTable* t) { (void)t; }
}
