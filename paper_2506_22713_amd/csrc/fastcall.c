/* CPython entry for eodabe_factor: the same C-ABI call as the ctypes binding,
 * with the argument conversion done in C (ctypes spends microseconds per
 * call on it, and a caller that factors matrices back to back pays that time
 * with the GPU idle, since every call ends with a stream sync).  The function
 * is reached through the address of eodabe_factor in the library the ctypes
 * binding has loaded (bind()), so one copy of the library serves both. */
#define PY_SSIZE_T_CLEAN
#include <Python.h>
#include <stdint.h>
#include <string.h>

#include "eodabe.h"

typedef int (*factor_fn)(eodabe_ctx*, const void*, int64_t, int64_t, int64_t, double, void*, size_t, void*,
                         void*, void*, int64_t, eodabe_info*);
static factor_fn g_factor = NULL;

/* bind(address of eodabe_factor) */
static PyObject* fc_bind(PyObject* self, PyObject* arg) {
  (void)self;
  void* p = PyLong_AsVoidPtr(arg);
  if (!p) {
    if (!PyErr_Occurred()) PyErr_SetString(PyExc_ValueError, "null function address");
    return NULL;
  }
  g_factor = (factor_fn)p;
  Py_RETURN_NONE;
}

/* factor(ctx, A, m, n, lda, tol, ws, ws_bytes, Ut, core, Vt, r_cap)
 *   -> (status, rank, blocks, status_flags, norm_a, eps, relres_est)
 * Pointers as Python ints (device addresses), sizes as ints; the GIL is
 * released for the call. */
static PyObject* fc_factor(PyObject* self, PyObject* const* args, Py_ssize_t nargs) {
  (void)self;
  if (!g_factor) {
    PyErr_SetString(PyExc_RuntimeError, "eodabe_factor not bound");
    return NULL;
  }
  if (nargs != 12) {
    PyErr_SetString(PyExc_TypeError, "factor() takes 12 arguments");
    return NULL;
  }
  eodabe_ctx* ctx = (eodabe_ctx*)PyLong_AsVoidPtr(args[0]);
  const void* A = PyLong_AsVoidPtr(args[1]);
  const int64_t m = PyLong_AsLongLong(args[2]), n = PyLong_AsLongLong(args[3]), lda = PyLong_AsLongLong(args[4]);
  const double tol = PyFloat_AsDouble(args[5]);
  void* ws = PyLong_AsVoidPtr(args[6]);
  const size_t wsb = PyLong_AsSize_t(args[7]);
  void* Ut = PyLong_AsVoidPtr(args[8]);
  void* core = PyLong_AsVoidPtr(args[9]);
  void* Vt = PyLong_AsVoidPtr(args[10]);
  const int64_t rc = PyLong_AsLongLong(args[11]);
  if (PyErr_Occurred()) return NULL;
  eodabe_info info;
  memset(&info, 0, sizeof(info));
  int st;
  Py_BEGIN_ALLOW_THREADS
  st = g_factor(ctx, A, m, n, lda, tol, ws, wsb, Ut, core, Vt, rc, &info);
  Py_END_ALLOW_THREADS
  return Py_BuildValue("(iLiiddd)", st, (long long)info.rank, info.blocks, info.status_flags, info.norm_a, info.eps,
                       info.relres_est);
}

static PyMethodDef fc_methods[] = {
    {"bind", (PyCFunction)fc_bind, METH_O, "bind(address of eodabe_factor)"},
    {"factor", (PyCFunction)(void (*)(void))fc_factor, METH_FASTCALL, "eodabe_factor with C-side marshalling"},
    {NULL, NULL, 0, NULL}};

static struct PyModuleDef fc_module = {PyModuleDef_HEAD_INIT, "_fastcall", NULL, -1, fc_methods, NULL, NULL, NULL,
                                       NULL};

PyMODINIT_FUNC PyInit__fastcall(void) { return PyModule_Create(&fc_module); }
