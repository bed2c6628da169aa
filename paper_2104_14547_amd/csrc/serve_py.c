/* CPython binding of the serving calls that run once per request
 * (nurbs_server_submit, nurbs_server_wait): argument marshalling only.
 * Buffers come in through the buffer protocol (C-contiguous float32), so a
 * request costs no ctypes conversions.  The library's entry points are bound
 * once, by address, from the already loaded libnurbsdiff. */
#define PY_SSIZE_T_CLEAN
#include <Python.h>
#include <stdint.h>
#include <string.h>

typedef int (*submit_fn)(void *, int, const float *, int, const float *, int, const float *, float *, double,
                         int64_t *);
typedef int (*wait_fn)(void *, int64_t, double *);

static submit_fn g_submit = NULL;
static wait_fn g_wait = NULL;

static PyObject *bind(PyObject *self, PyObject *args) {
    unsigned long long s, w;
    if (!PyArg_ParseTuple(args, "KK", &s, &w)) return NULL;
    g_submit = (submit_fn)(uintptr_t)s;
    g_wait = (wait_fn)(uintptr_t)w;
    Py_RETURN_NONE;
}

/* Gets a C-contiguous float32 buffer of obj (writable if asked). */
static int f32_buffer(PyObject *obj, Py_buffer *v, int writable, const char *name) {
    int flags = PyBUF_C_CONTIGUOUS | PyBUF_FORMAT | (writable ? PyBUF_WRITABLE : 0);
    if (PyObject_GetBuffer(obj, v, flags) != 0) return -1;
    if (v->itemsize != 4 || !v->format || strcmp(v->format, "f") != 0) {
        PyBuffer_Release(v);
        PyErr_Format(PyExc_TypeError, "%s must be a contiguous float32 array", name);
        return -1;
    }
    return 0;
}

/* submit(handle, surf, us, vs, target, out, t_arrival) -> (status, id) */
static PyObject *submit(PyObject *self, PyObject *args) {
    unsigned long long h;
    int surf;
    PyObject *ou, *ov, *ot, *oo;
    double t;
    if (!PyArg_ParseTuple(args, "KiOOOOd", &h, &surf, &ou, &ov, &ot, &oo, &t)) return NULL;
    if (!g_submit) {
        PyErr_SetString(PyExc_RuntimeError, "serving calls not bound");
        return NULL;
    }
    Py_buffer bu, bv, bt, bo;
    if (f32_buffer(ou, &bu, 0, "us")) return NULL;
    if (f32_buffer(ov, &bv, 0, "vs")) {
        PyBuffer_Release(&bu);
        return NULL;
    }
    if (f32_buffer(ot, &bt, 0, "target")) {
        PyBuffer_Release(&bu);
        PyBuffer_Release(&bv);
        return NULL;
    }
    if (f32_buffer(oo, &bo, 1, "out")) {
        PyBuffer_Release(&bu);
        PyBuffer_Release(&bv);
        PyBuffer_Release(&bt);
        return NULL;
    }
    const Py_ssize_t nu = bu.len / 4, nv = bv.len / 4;
    int rc;
    int64_t id = -1;
    if (nu > 65535 || nv > 65535 || bt.len / 4 != 3 * nu * nv) {
        rc = -1; /* NURBS_EINVAL */
    } else {
        Py_BEGIN_ALLOW_THREADS
        rc = g_submit((void *)(uintptr_t)h, surf, (const float *)bu.buf, (int)nu, (const float *)bv.buf, (int)nv,
                      (const float *)bt.buf, (float *)bo.buf, t, &id);
        Py_END_ALLOW_THREADS
    }
    PyBuffer_Release(&bu);
    PyBuffer_Release(&bv);
    PyBuffer_Release(&bt);
    PyBuffer_Release(&bo);
    return Py_BuildValue("iL", rc, (long long)id);
}

/* wait(handle, id) -> (status, latency seconds); releases the interpreter lock */
static PyObject *wait_req(PyObject *self, PyObject *args) {
    unsigned long long h;
    long long id;
    if (!PyArg_ParseTuple(args, "KL", &h, &id)) return NULL;
    if (!g_wait) {
        PyErr_SetString(PyExc_RuntimeError, "serving calls not bound");
        return NULL;
    }
    double lat = 0.0;
    int rc;
    Py_BEGIN_ALLOW_THREADS
    rc = g_wait((void *)(uintptr_t)h, (int64_t)id, &lat);
    Py_END_ALLOW_THREADS
    return Py_BuildValue("id", rc, lat);
}

static PyMethodDef methods[] = {
    {"bind", bind, METH_VARARGS, "bind(submit_address, wait_address)"},
    {"submit", submit, METH_VARARGS, "submit(handle, surf, us, vs, target, out, t_arrival) -> (status, id)"},
    {"wait", wait_req, METH_VARARGS, "wait(handle, id) -> (status, latency)"},
    {NULL, NULL, 0, NULL},
};

static struct PyModuleDef module = {PyModuleDef_HEAD_INIT, "_serve_py", NULL, -1, methods};

PyMODINIT_FUNC PyInit__serve_py(void) { return PyModule_Create(&module); }
