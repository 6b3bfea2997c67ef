/* A Python interpreter linked with the AddressSanitizer and
 * UndefinedBehaviorSanitizer runtimes, so that the host-instrumented copy of
 * libpeifem.so can be loaded into the test suite: the runtime sits in the
 * executable itself, ahead of every library the process loads.  Device code
 * is not instrumented. */
#include <Python.h>

int main(int argc, char **argv) { return Py_BytesMain(argc, argv); }
