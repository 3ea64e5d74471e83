// Edge-coefficient classes: the per-edge material rule (Sec. 3) and the theta
// coefficients of Algorithm 1 step 3 evaluated once per distinct combination
// of the four cells sharing an edge, instead of once per edge per step.
//
// Built on the host from a copy of the bound maps: every distinct cell
// material (eps_r, sigma, inv_lambda2, compared bit for bit) gets a 16-bit id,
// every distinct ordered 4-tuple of ids around an edge gets a class, and a
// device kernel turns each class's tuple into (ca, cb, cj) with the same code
// the sweeps run on the maps.
#include <cstring>
#include <vector>

#include "sim_internal.h"

using namespace tfl;
using namespace tfl::detail;

namespace {

constexpr int kMaxCellMaterials = 65536;

// Open-addressing index of keys of W 64-bit words (ids 0, 1, ... in order of
// first insertion), with room for `limit` keys at a load factor below 1/4.
template <int W>
class KeyIndex {
  public:
    explicit KeyIndex(int limit) : limit_(limit)
    {
        size_t cap = 1;
        while (cap < 4 * (size_t)limit) cap <<= 1;
        mask_ = cap - 1;
        keys_.resize(cap * W);
        ids_.assign(cap, -1);
    }
    // Id of `key`, adding it if new; -1 when the index already holds `limit` keys.
    int find_or_add(const uint64_t *key)
    {
        uint64_t h = 0x9e3779b97f4a7c15ull;
        for (int w = 0; w < W; ++w) h = mix(h ^ key[w]);
        for (size_t slot = h & mask_;; slot = (slot + 1) & mask_) {
            const int id = ids_[slot];
            if (id < 0) {
                if (count_ == limit_) return -1;
                std::memcpy(&keys_[slot * W], key, W * sizeof(uint64_t));
                ids_[slot] = count_;
                return count_++;
            }
            if (std::memcmp(&keys_[slot * W], key, W * sizeof(uint64_t)) == 0) return id;
        }
    }
    int count() const { return count_; }

  private:
    static uint64_t mix(uint64_t x)  // splitmix64 finaliser
    {
        x ^= x >> 30;
        x *= 0xbf58476d1ce4e5b9ull;
        x ^= x >> 27;
        x *= 0x94d049bb133111ebull;
        return x ^ (x >> 31);
    }
    int limit_, count_ = 0;
    size_t mask_;
    std::vector<uint64_t> keys_;
    std::vector<int> ids_;
};

template <typename T>
uint64_t bits(T v)
{
    if constexpr (sizeof(T) == 8) {
        uint64_t b;
        std::memcpy(&b, &v, 8);
        return b;
    } else {
        uint32_t b;
        std::memcpy(&b, &v, 4);
        return b;
    }
}

struct ClassLayout {
    size_t cls_bytes;    // one class array (N uint16, padded)
    size_t table_off;    // TFL_MAX_EDGE_CLASSES x 4 values
    size_t mat_off;      // staging: kMaxCellMaterials x 3 values
    size_t tuple_off;    // staging: TFL_MAX_EDGE_CLASSES uint64
    size_t total;
};

ClassLayout class_layout(const tfl_sim *s)
{
    ClassLayout L;
    L.cls_bytes = round256((size_t)s->N * sizeof(uint16_t));
    L.table_off = 3 * L.cls_bytes;
    L.mat_off = L.table_off + round256((size_t)TFL_MAX_EDGE_CLASSES * 4 * s->esz);
    L.tuple_off = L.mat_off + round256((size_t)kMaxCellMaterials * 3 * s->esz);
    L.total = L.tuple_off + round256((size_t)TFL_MAX_EDGE_CLASSES * sizeof(uint64_t));
    return L;
}

template <typename T>
int build_classes(tfl_sim *s, void *buf, int *ncls_out, hipStream_t st)
{
    const long long N = s->N;
    const int nx = (int)s->cfg.nx, ny = (int)s->cfg.ny, nz = (int)s->cfg.nz;
    const long long sxy = (long long)nx * ny;
    std::vector<T> eps(N), sig(N), ell(N);
    hipError_t e = hipMemcpyAsync(eps.data(), s->eps, N * sizeof(T), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(sig.data(), s->sig, N * sizeof(T), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ell.data(), s->ell, N * sizeof(T), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(s, e, "edge classes: map readback");

    // cell material ids (runs of equal cells along x skip the lookup)
    std::vector<uint16_t> cid(N);
    std::vector<T> mat;
    KeyIndex<3> cells(kMaxCellMaterials);
    uint64_t prev[3] = {~0ull, ~0ull, ~0ull};
    int prev_id = -1;
    for (long long c = 0; c < N; ++c) {
        const uint64_t key[3] = {bits(eps[c]), bits(sig[c]), bits(ell[c])};
        if (prev_id < 0 || key[0] != prev[0] || key[1] != prev[1] || key[2] != prev[2]) {
            const int before = cells.count();
            prev_id = cells.find_or_add(key);
            if (prev_id < 0)
                return fail(s, TFL_E_RANGE, "edge classes: more than %d distinct cell materials", kMaxCellMaterials);
            if (prev_id == before) {
                mat.push_back(eps[c]);
                mat.push_back(sig[c]);
                mat.push_back(ell[c]);
            }
            std::memcpy(prev, key, sizeof(prev));
        }
        cid[c] = (uint16_t)prev_id;
    }
    eps = std::vector<T>();
    sig = std::vector<T>();
    ell = std::vector<T>();

    // classes: the ordered ids of the four cells of each edge, in the order the sweeps pass them to
    // the edge rule.  x edge of cell (i,j,k): (i,j,k), (i,j,k-1), (i,j-1,k), (i,j-1,k-1); y edge:
    // (i,j,k), (i-1,j,k), (i,j,k-1), (i-1,j,k-1); z edge: (i,j,k), (i,j-1,k), (i-1,j,k), (i-1,j-1,k);
    // indices wrap as in the sweeps (the wall edges of CPML axes are zeroed there regardless).
    std::vector<uint16_t> cls(3 * (size_t)N);
    std::vector<uint64_t> tuples;
    KeyIndex<1> classes(TFL_MAX_EDGE_CLASSES);
    for (int ax = 0; ax < 3; ++ax) {
        uint16_t *out = cls.data() + (size_t)ax * N;
        uint64_t prev_key = ~0ull;
        int prev_cls = -1;
        for (int k = 0; k < nz; ++k) {
            const int km = (k == 0) ? nz - 1 : k - 1;
            for (int j = 0; j < ny; ++j) {
                const int jm = (j == 0) ? ny - 1 : j - 1;
                const long long r = (long long)k * sxy + (long long)j * nx;
                const long long rz = (long long)km * sxy + (long long)j * nx;
                const long long ry = (long long)k * sxy + (long long)jm * nx;
                const long long ryz = (long long)km * sxy + (long long)jm * nx;
                for (int i = 0; i < nx; ++i) {
                    const int im = (i == 0) ? nx - 1 : i - 1;
                    uint64_t q0 = cid[r + i], q1, q2, q3;
                    if (ax == 0) {
                        q1 = cid[rz + i]; q2 = cid[ry + i]; q3 = cid[ryz + i];
                    } else if (ax == 1) {
                        q1 = cid[r + im]; q2 = cid[rz + i]; q3 = cid[rz + im];
                    } else {
                        q1 = cid[ry + i]; q2 = cid[r + im]; q3 = cid[ry + im];
                    }
                    const uint64_t key = q0 | (q1 << 16) | (q2 << 32) | (q3 << 48);
                    if (key != prev_key || prev_cls < 0) {
                        const int before = classes.count();
                        prev_cls = classes.find_or_add(&key);
                        if (prev_cls < 0)
                            return fail(s, TFL_E_RANGE, "edge classes: more than %d distinct edge materials",
                                        TFL_MAX_EDGE_CLASSES);
                        if (prev_cls == before) tuples.push_back(key);
                        prev_key = key;
                    }
                    out[r + i] = (uint16_t)prev_cls;
                }
            }
        }
    }

    const ClassLayout L = class_layout(s);
    char *b = (char *)buf;
    const int ncls = classes.count();
    e = hipMemcpyAsync(b + L.mat_off, mat.data(), mat.size() * sizeof(T), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b + L.tuple_off, tuples.data(), tuples.size() * sizeof(uint64_t), hipMemcpyHostToDevice, st);
    for (int ax = 0; ax < 3 && e == hipSuccess; ++ax)
        e = hipMemcpyAsync(b + ax * L.cls_bytes, cls.data() + (size_t)ax * N, N * sizeof(uint16_t),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_class_table<T>(make_args<T>(s), (const T *)(b + L.mat_off), (const uint64_t *)(b + L.tuple_off),
                                  ncls, (T *)(b + L.table_off), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(s, e, "edge classes: upload");
    *ncls_out = ncls;
    return TFL_OK;
}

}  // namespace

namespace tfl {
namespace detail {

void class_pointers(const tfl_sim *s, const uint16_t *cls[3], const void **table)
{
    if (!s->cls) {
        cls[0] = cls[1] = cls[2] = nullptr;
        *table = nullptr;
        return;
    }
    const ClassLayout L = class_layout(s);
    const char *b = (const char *)s->cls;
    for (int ax = 0; ax < 3; ++ax) cls[ax] = (const uint16_t *)(b + ax * L.cls_bytes);
    *table = b + L.table_off;
}

}  // namespace detail
}  // namespace tfl

int tfl_edge_class_bytes(const tfl_sim *s, size_t *bytes)
{
    if (!s || !bytes) return fail(nullptr, TFL_E_INVAL, "null argument");
    *bytes = class_layout(s).total;
    return TFL_OK;
}

int tfl_bind_edge_classes(tfl_sim *s, void *buffer, int *nclasses, void *stream)
{
    if (!s) return fail(nullptr, TFL_E_INVAL, "null handle");
    s->cls = nullptr;
    s->ncls = 0;
    if (nclasses) *nclasses = 0;
    if (!buffer) return TFL_OK;
    if (!aligned(buffer)) return fail(s, TFL_E_INVAL, "class buffer must be 256-byte aligned");
    if (!s->maps_bound) return fail(s, TFL_E_STATE, "materials not bound (tfl_bind_materials)");
    int ncls = 0;
    const int rc = s->esz == 8 ? build_classes<double>(s, buffer, &ncls, (hipStream_t)stream)
                               : build_classes<float>(s, buffer, &ncls, (hipStream_t)stream);
    if (rc != TFL_OK) return rc;
    s->cls = buffer;
    s->ncls = ncls;
    if (nclasses) *nclasses = ncls;
    return TFL_OK;
}
