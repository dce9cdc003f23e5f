// Five-qubit GHZ state over two quantum registers, then every qubit measured.
OPENQASM 2.0;
include "qelib1.inc";
qreg a[2];
qreg b[3];
creg m[5];
h a[0];
cx a[0], a[1];
cx a[1], b[0];
cx b[0], b[1];
cx b[1], b[2];
barrier a, b;
measure a[0] -> m[0];
measure a[1] -> m[1];
measure b[0] -> m[2];
measure b[1] -> m[3];
measure b[2] -> m[4];
